"""Literal 1D scheme of the paper in numpy (test infrastructure only).

A second, independent transcription of the one-dimensional method, used to
pin the 2D oracle: a y-uniform 2D run must reproduce it.  It follows the 1D
formulas as printed, vectorised over cells and faces:

* eq. (SW1Dscheme), Section 3.1:
  U*_i = U^n_i - dt/dx [F_{i+1/2L} - F_{i-1/2R} - Fc_i];
* hydrostatic reconstruction, S_{i+1/2L}, S_{i-1/2R} and Fc_i, Section 3.1;
* HLL flux with c1 = min over U_L, U_R of u - sqrt(gh) and c2 = max of
  u + sqrt(gh), Section 3.3 (or the Rusanov flux, another consistent flux
  that section names, or the VFRoe-ncv flux Section 4.1 lists: the
  interface state of the Riemann problem in the variables (2 sqrt(gh), u)
  linearized about the mean state);
* MUSCL with minmod on h, h+z and u and the modified velocity, Section 3.4,
  written with divided differences exactly as printed (or ENO: the
  one-sided slope of smaller magnitude, none in a dry cell; modified ENO:
  the same with the depth slope limited to 2 h / dx in magnitude);
* semi-implicit friction and Heun's method, Section 3.2;
* first order (Section 3.3): no reconstruction (zero slopes) and one
  explicit Euler stage per step.

Two ghost cells per side (wall: mirror with negated discharge; outflow:
copy of the boundary cell).  The dry threshold h_eps and the Manning split
are the same readings as the 2D oracle's.
"""

from __future__ import annotations

import numpy as np

WALL, OUTFLOW = 0, 1


def _ghost(a, bc_w, bc_e, odd):
    """Pad a 1D array with two ghost cells per side."""
    w = a[[1, 0]] if bc_w == WALL else a[[0, 0]]
    e = a[[-1, -2]] if bc_e == WALL else a[[-1, -1]]
    if odd:
        if bc_w == WALL:
            w = -w
        if bc_e == WALL:
            e = -e
    return np.concatenate([w, a, e])


def _minmod(x, y):
    out = np.zeros_like(x)
    pos = (x >= 0) & (y >= 0)
    neg = (x <= 0) & (y <= 0)
    out[pos] = np.minimum(x[pos], y[pos])
    out[neg & ~pos] = np.maximum(x[neg & ~pos], y[neg & ~pos])
    return out


def _eno(x, y):
    """The argument of smaller magnitude (the first on ties)."""
    return np.where(np.abs(x) <= np.abs(y), x, y)


def _vfroe(hL, uL, hR, uR, g):
    """Mass and momentum flux of the state at x/t = 0 of the Riemann problem
    of (2c, u), c = sqrt(gh), linearized about the mean state."""
    wl, wr = hL > 0, hR > 0
    uL = np.where(wl, uL, uR)
    uR = np.where(wr, uR, uL)
    cL, cR = np.sqrt(g * hL), np.sqrt(g * hR)
    um, cm = (uL + uR) / 2, (cL + cR) / 2
    # subsonic interface: 2c + u from the left, 2c - u from the right
    cs = np.maximum(cm + (uL - uR) / 4, 0.0)
    us = um + (cL - cR)
    h = np.where(um - cm >= 0, hL, np.where(um + cm <= 0, hR, cs * cs / g))
    u = np.where(um - cm >= 0, uL, np.where(um + cm <= 0, uR, us))
    both_dry = ~wl & ~wr
    F0 = np.where(both_dry, 0.0, h * u)
    F1 = np.where(both_dry, 0.0, h * u * u + g * h * h / 2)
    return F0, F1


def convective_rate(h, q, z, dx, g, h_eps, bc, order=2, flux="hll", recon="minmod"):
    """Returns the bracket [F_{i+1/2L} - F_{i-1/2R} - Fc_i] and max speed."""
    hp = _ghost(h, bc[0], bc[1], False)
    qp = _ghost(q, bc[0], bc[1], True)
    zp = _ghost(z, bc[0], bc[1], False)
    wet = hp > h_eps
    u = np.where(wet, qp / np.where(wet, hp, 1.0), 0.0)
    eta = hp + zp
    # cells -1..n  (padded indices 1..n+2)
    c = slice(1, -1)
    lo = slice(0, -2)
    hi = slice(2, None)
    lim = _minmod if recon == "minmod" else _eno
    Dh = lim((hp[c] - hp[lo]) / dx, (hp[hi] - hp[c]) / dx)
    De = lim((eta[c] - eta[lo]) / dx, (eta[hi] - eta[c]) / dx)
    Du = lim((u[c] - u[lo]) / dx, (u[hi] - u[c]) / dx)
    if recon in ("eno", "enomod"):
        # a dry cell is not reconstructed
        dry = hp[c] <= h_eps
        Dh, De, Du = (np.where(dry, 0.0, D) for D in (Dh, De, Du))
    if recon == "enomod":
        # face depths h -/+ dx/2 Dh within [0, 2h]
        Dh = np.clip(Dh, -2 * hp[c] / dx, 2 * hp[c] / dx)
    if order == 1:
        Dh, De, Du = np.zeros_like(Dh), np.zeros_like(De), np.zeros_like(Du)
    h_m = hp[c] - dx / 2 * Dh           # h_{i-1/2+}
    h_p = hp[c] + dx / 2 * Dh           # h_{i+1/2-}
    z_m = (eta[c] - dx / 2 * De) - h_m
    z_p = (eta[c] + dx / 2 * De) - h_p
    hc = hp[c]
    wc = hc > h_eps
    hs = np.where(wc, hc, 1.0)
    u_m = np.where(wc, u[c] - h_p / hs * dx / 2 * Du, u[c])
    u_p = np.where(wc, u[c] + h_m / hs * dx / 2 * Du, u[c])
    # faces between reconstructed cells k and k+1 (k = -1..n-1)
    hm_, zm_, um_ = h_p[:-1], z_p[:-1], u_p[:-1]   # left state  (U_-, z_-)
    hq_, zq_, uq_ = h_m[1:], z_m[1:], u_m[1:]       # right state (U_+, z_+)
    zs = np.maximum(zm_, zq_)
    hL = np.maximum(hm_ + zm_ - zs, 0.0)
    hR = np.maximum(hq_ + zq_ - zs, 0.0)
    cL = np.sqrt(g * hL)
    cR = np.sqrt(g * hR)
    c1 = np.minimum(um_ - cL, uq_ - cR)
    c2 = np.maximum(um_ + cL, uq_ + cR)
    FL0, FL1 = hL * um_, hL * um_ * um_ + g * hL * hL / 2
    FR0, FR1 = hR * uq_, hR * uq_ * uq_ + g * hR * hR / 2
    if flux == "vfroe":
        F0, F1 = _vfroe(hL, um_, hR, uq_, g)
    elif flux == "rusanov":
        # local Lax-Friedrichs: (F(U_L) + F(U_R))/2 - c/2 (U_R - U_L)
        c = np.maximum(np.abs(um_) + cL, np.abs(uq_) + cR)
        F0 = (FL0 + FR0) / 2 - c / 2 * (hR - hL)
        F1 = (FL1 + FR1) / 2 - c / 2 * (hR * uq_ - hL * um_)
    else:
        den = np.where((c1 < 0) & (c2 > 0), c2 - c1, 1.0)
        mid0 = (c2 * FL0 - c1 * FR0) / den + c1 * c2 / den * (hR - hL)
        mid1 = (c2 * FL1 - c1 * FR1) / den + c1 * c2 / den * (hR * uq_ - hL * um_)
        F0 = np.where(c1 >= 0, FL0, np.where(c2 <= 0, FR0, mid0))
        F1 = np.where(c1 >= 0, FL1, np.where(c2 <= 0, FR1, mid1))
    SL = g * (hm_ ** 2 - hL ** 2) / 2   # S_{i+1/2L}, momentum component
    SR = g * (hq_ ** 2 - hR ** 2) / 2   # S_{i+1/2R}
    speed = np.maximum(np.abs(um_) + np.sqrt(g * hm_),
                       np.abs(uq_) + np.sqrt(g * hq_)).max()
    # cells 0..n-1 : right face index k+1, left face index k
    hm_c, hp_c = h_m[1:-1], h_p[1:-1]
    zm_c, zp_c = z_m[1:-1], z_p[1:-1]
    Fc1 = -g * (hm_c + hp_c) / 2 * (zp_c - zm_c)
    B0 = F0[1:] - F0[:-1]
    B1 = (F1[1:] + SL[1:]) - (F1[:-1] + SR[:-1]) - Fc1
    return B0, B1, speed


def friction(h0, q0, h1, q1, dt, law, coef, g, h_eps):
    q1 = np.where(h1 <= h_eps, 0.0, q1)
    if law == 0:
        return q1
    act = (h1 > h_eps) & (h0 > h_eps)
    h0s = np.where(act, h0, 1.0)
    h1s = np.where(act, h1, 1.0)
    if law == 2:
        den = 1 + dt * coef / 8 * np.abs(q0) / (h0s * h1s)
    else:
        den = 1 + dt * g * coef ** 2 * np.abs(q0) / (h0s * h1s ** (4.0 / 3.0))
    return np.where(act, q1 / den, q1)


def heun_step(h, q, z, dt, dx, g=9.81, h_eps=1e-12, bc=(WALL, WALL), law=0,
              coef=0.0, flux="hll", recon="minmod"):
    def phi_stage(hh, qq):
        B0, B1, _ = convective_rate(hh, qq, z, dx, g, h_eps, bc, flux=flux, recon=recon)
        h1 = hh - dt / dx * B0
        q1 = qq - dt / dx * B1
        q1 = friction(hh, qq, h1, q1, dt, law, coef, g, h_eps)
        return h1, q1

    h1, q1 = phi_stage(h, q)
    h2, q2 = phi_stage(h1, q1)
    return (h + h2) / 2, (q + q2) / 2


def euler_step(h, q, z, dt, dx, g=9.81, h_eps=1e-12, bc=(WALL, WALL), law=0, coef=0.0):
    """First order: U^{n+1} = friction(U^n + dt Phi_1(U^n))."""
    B0, B1, _ = convective_rate(h, q, z, dx, g, h_eps, bc, order=1)
    h1 = h - dt / dx * B0
    q1 = q - dt / dx * B1
    return h1, friction(h, q, h1, q1, dt, law, coef, g, h_eps)


def cfl_dt(h, q, z, dx, cfl=0.5, g=9.81, h_eps=1e-12, bc=(WALL, WALL)):
    """eq. (cfl) on the reconstructed states (1D)."""
    _, _, speed = convective_rate(h, q, z, dx, g, h_eps, bc)
    return cfl * dx / speed
