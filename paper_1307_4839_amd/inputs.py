"""Seeded synthetic workloads for the 2D shallow-water step.

This module builds inputs only: terrains (DEMs), initial states, friction
fields, gauge positions and the scalar parameters of each workload.  It holds
none of the numerical scheme.  Both the CPU oracle (``oracle/``) and the HIP
library consume exactly the arrays produced here.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).  Arrays
are float64, shape ``[ny, nx]``, row-major with x fastest.  Cell centres are
``x_i = (i + 1/2) dx`` and ``y_j = (j + 1/2) dy``.

Workload recipes (they stand in for the paper's Malpasset valley, Section 4.2,
and its 5120 x 5120 scaling run, Section 6.3, whose DEMs are not available):

* ``dam_break_200``: 200 x 200, dx = 1 m; plane of slope 0.005 falling towards
  +x plus 5 Gaussian bumps (0.5 m, sigma 10 m); 2 m of water for x < 100 m;
  Manning n = 0.03; walls on all sides; run to t = 30 s.
* ``valley_2048``: 2048 x 2048, dx = 5 m; V-shaped valley (side slope 0.2,
  longitudinal slope 0.003 falling towards +y) plus 3 m of 4-octave Perlin fBm
  (base wavelength 1280 m); reservoir at a 50 m level in rows j < 300, dry
  below; Manning n = 0.033; free outflow at the north (downstream) edge.
* ``hillslope_8192``: 8192 x 8192, dx = 1 m; plane of slope 0.02 falling
  towards +x plus 0.3 m of fBm (base wavelength 64 m); initially dry; rain
  50 mm/h; Green-Ampt Ks = 1e-6 m/s, suction 0.1 m, porosity 0.4 (initial
  moisture 0); Darcy-Weisbach f = 0.3; free outflow at the east (downslope)
  edge, walls elsewhere; dt_max = 1 s.
* ``ensemble``: scenario k of 256 uses seed 4000 + k; square grids with
  n = round(exp(U(ln 64, ln 1024))), dx = 2 m; slope U(0.005, 0.05) towards
  +x plus 1 m fBm; dry; rain U(10, 100) mm/h; Manning U(0.02, 0.06); free
  outflow at the east edge; dt_max = 1 s.
* ``calibration_1024``: 1024 x 1024, dx = 2 m; the valley recipe scaled to
  2048 m with a dam at row 150; Manning field 0.03 (1 + 0.2 xi) with xi a
  Gaussian-filtered (sigma 20 cells) white noise scaled to max|xi| = 1;
  64 gauges on the valley floor (|x - xc| <= 40 m, rows 150..600).

Any size can be requested through the ``nx``/``ny`` arguments so that tests
can run the same recipe at small sizes.
"""

from __future__ import annotations

import dataclasses
import math
import os
from typing import Dict, Optional

import numpy as np

WALL = 0
OUTFLOW = 1
IMPOSED_H = 2   # depth imposed (Riemann invariant for the velocity)
IMPOSED_Q = 3   # inflow discharge imposed (Riemann invariant for the depth)
IMPOSED_HQ = 4  # both (supercritical inflow)

FRIC_NONE = 0
FRIC_MANNING = 1
FRIC_DARCY = 2

MM_PER_HOUR = 1.0 / 3.6e6  # m/s per mm/h


@dataclasses.dataclass
class Workload:
    """A complete initial-value problem: scalar parameters plus arrays."""

    name: str
    nx: int
    ny: int
    dx: float
    dy: float
    z: np.ndarray
    h: np.ndarray
    qx: np.ndarray
    qy: np.ndarray
    bc: tuple = (WALL, WALL, WALL, WALL)  # west, east, south, north
    bc_h: tuple = (0.0, 0.0, 0.0, 0.0)    # imposed depth per side [m]
    bc_q: tuple = (0.0, 0.0, 0.0, 0.0)    # imposed inflow discharge per side [m^2/s]
    g: float = 9.81
    cfl: float = 0.5
    dt_max: float = math.inf
    dt_min: float = 0.0  # a CFL dt below it (not clipped to t_end) stops the run
    h_eps: float = 1e-12
    fric_law: int = FRIC_NONE
    fric_coef: float = 0.0
    fric: Optional[np.ndarray] = None  # per-cell coefficient field
    rain: float = 0.0  # m/s
    infil_on: int = 0
    ks: float = 0.0
    psi: float = 0.0
    dtheta: float = 0.0
    vinf: Optional[np.ndarray] = None
    # rain R(t, x, y) = r(t) w(x, y): piecewise-constant hyetograph r (values
    # rain_r [m/s] from breakpoints rain_t [s]; `rain` when absent) and a
    # per-cell weight w (1 when absent)
    rain_t: Optional[np.ndarray] = None
    rain_r: Optional[np.ndarray] = None
    rain_w: Optional[np.ndarray] = None
    # per-cell Green-Ampt parameters (the scalars when absent)
    ks_f: Optional[np.ndarray] = None
    psi_f: Optional[np.ndarray] = None
    dtheta_f: Optional[np.ndarray] = None
    # 2: MUSCL + Heun (the paper's scheme); 1: first order (piecewise
    # constant, one Euler stage; the paper uses n_CFL = 1 with it)
    order: int = 2
    # numerical flux: 0 HLL (the paper's), 1 Rusanov, 2 kinetic, 3 VFRoe-ncv
    flux: int = 0
    # second-order reconstruction: 0 MUSCL (the paper's), 1 ENO, 2 modified ENO
    recon: int = 0
    t_end: float = math.inf
    nsteps: int = 0
    gauges: Optional[np.ndarray] = None  # flat cell indices
    extra: Dict[str, object] = dataclasses.field(default_factory=dict)

    def params(self) -> Dict[str, object]:
        return dict(nx=self.nx, ny=self.ny, dx=self.dx, dy=self.dy, g=self.g,
                    cfl=self.cfl, dt_max=self.dt_max, h_eps=self.h_eps,
                    bc=tuple(self.bc), fric_law=self.fric_law,
                    fric_coef=self.fric_coef, rain=self.rain,
                    infil_on=self.infil_on, ks=self.ks, psi=self.psi,
                    dtheta=self.dtheta, order=self.order, flux=self.flux,
                    bc_h=tuple(self.bc_h), bc_q=tuple(self.bc_q), dt_min=self.dt_min,
                    recon=self.recon)

    def copy(self) -> "Workload":
        out = dataclasses.replace(self)
        for f in ("z", "h", "qx", "qy", "fric", "vinf", "gauges", "rain_t", "rain_r",
                  "rain_w", "ks_f", "psi_f", "dtheta_f"):
            a = getattr(self, f)
            if a is not None:
                setattr(out, f, a.copy())
        out.extra = dict(self.extra)
        return out


# ----------------------------------------------------------------------------
# Terrain noise
# ----------------------------------------------------------------------------

class _Perlin:
    """Classic 2D gradient noise with the quintic fade 6t^5 - 15t^4 + 10t^3.

    A seeded permutation of 0..255 hashes lattice points onto 256 seeded unit
    gradient vectors.
    """

    def __init__(self, rng: np.random.Generator):
        perm = rng.permutation(256)
        self.perm = np.concatenate([perm, perm]).astype(np.int64)
        ang = rng.uniform(0.0, 2.0 * math.pi, 256)
        self.gx = np.cos(ang)
        self.gy = np.sin(ang)

    @staticmethod
    def _fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    def __call__(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        x0 = np.floor(x)
        y0 = np.floor(y)
        fx = x - x0
        fy = y - y0
        xi = x0.astype(np.int64) & 255
        yi = y0.astype(np.int64) & 255
        p = self.perm
        h00 = p[p[xi] + yi]
        h10 = p[p[xi + 1] + yi]
        h01 = p[p[xi] + yi + 1]
        h11 = p[p[xi + 1] + yi + 1]
        n00 = self.gx[h00] * fx + self.gy[h00] * fy
        n10 = self.gx[h10] * (fx - 1.0) + self.gy[h10] * fy
        n01 = self.gx[h01] * fx + self.gy[h01] * (fy - 1.0)
        n11 = self.gx[h11] * (fx - 1.0) + self.gy[h11] * (fy - 1.0)
        sx = self._fade(fx)
        sy = self._fade(fy)
        a = n00 + sx * (n10 - n00)
        b = n01 + sx * (n11 - n01)
        return a + sy * (b - a)


def fbm(rng: np.random.Generator, nx: int, ny: int, dx: float, dy: float,
        wavelength: float, octaves: int = 4, lacunarity: float = 2.0,
        persistence: float = 0.5, chunk_rows: int = 256) -> np.ndarray:
    """Fractal Brownian motion of Perlin noise normalised to max|.| = 1.

    Row chunks are evaluated on a thread pool (numpy releases the GIL); the
    values do not depend on the chunking or the thread count.
    """
    noise = _Perlin(rng)
    offs = rng.uniform(0.0, 256.0, size=(octaves, 2))
    xs = (np.arange(nx) + 0.5) * dx
    out = np.empty((ny, nx), dtype=np.float64)

    def work(r0):
        r1 = min(ny, r0 + chunk_rows)
        ys = (np.arange(r0, r1) + 0.5) * dy
        X, Y = np.meshgrid(xs, ys)
        acc = np.zeros_like(X)
        amp, freq = 1.0, 1.0 / wavelength
        for o in range(octaves):
            acc += amp * noise(X * freq + offs[o, 0], Y * freq + offs[o, 1])
            amp *= persistence
            freq *= lacunarity
        out[r0:r1] = acc

    starts = list(range(0, ny, chunk_rows))
    if len(starts) > 1:
        from concurrent.futures import ThreadPoolExecutor
        nthreads = min(len(starts), max(1, min(16, os.cpu_count() or 1)))
        with ThreadPoolExecutor(nthreads) as ex:
            list(ex.map(work, starts))
    else:
        work(0)
    m = np.abs(out).max()
    if m > 0:
        out /= m
    return out


def _centres(n: int, d: float) -> np.ndarray:
    return (np.arange(n) + 0.5) * d


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

def dam_break_200(nx: int = 200, ny: int = 200, seed: int = 1) -> Workload:
    rng = np.random.default_rng(seed)
    dx = dy = 1.0
    Lx, Ly = nx * dx, ny * dy
    x = _centres(nx, dx)[None, :]
    y = _centres(ny, dy)[:, None]
    z = 0.005 * (Lx - x) + np.zeros((ny, 1))
    centres = rng.uniform(0.0, 1.0, size=(5, 2)) * np.array([Lx, Ly])
    for cx, cy in centres:
        r2 = (x - cx) ** 2 + (y - cy) ** 2
        z = z + 0.5 * np.exp(-r2 / (2.0 * 10.0 ** 2))
    h = np.where(x < 0.5 * Lx, 2.0, 0.0) + np.zeros((ny, 1))
    zero = np.zeros((ny, nx))
    return Workload("dam_break_200", nx, ny, dx, dy, z=np.ascontiguousarray(z),
                    h=np.ascontiguousarray(h), qx=zero.copy(), qy=zero.copy(),
                    bc=(WALL, WALL, WALL, WALL), fric_law=FRIC_MANNING,
                    fric_coef=0.03, t_end=30.0, nsteps=100000)


def _valley(rng, nx, ny, d, side, slope, noise_amp, wavelength):
    Lx, Ly = nx * d, ny * d
    x = _centres(nx, d)[None, :]
    y = _centres(ny, d)[:, None]
    xc = 0.5 * Lx
    z = side * np.abs(x - xc) + slope * (Ly - y)
    z = z + noise_amp * fbm(rng, nx, ny, d, d, wavelength)
    return z, x, y, xc


def valley_2048(nx: int = 2048, ny: int = 2048, seed: int = 2,
                dam_row: int = 300) -> Workload:
    rng = np.random.default_rng(seed)
    d = 5.0
    z, x, y, xc = _valley(rng, nx, ny, d, 0.2, 0.003, 3.0, 1280.0)
    rows = np.arange(ny)[:, None]
    h = np.where(rows < dam_row, np.maximum(50.0 - z, 0.0), 0.0)
    zero = np.zeros((ny, nx))
    return Workload("valley_2048", nx, ny, d, d, z=z, h=np.ascontiguousarray(h),
                    qx=zero.copy(), qy=zero.copy(),
                    bc=(WALL, WALL, WALL, OUTFLOW), fric_law=FRIC_MANNING,
                    fric_coef=0.033, nsteps=2000)


def valley_5120(nx: int = 5120, ny: int = 5120, seed: int = 6,
                dam_row: int = 750) -> Workload:
    """The valley of valley_2048 (same 10.24 km extent, side slopes, down-valley
    slope, 1280 m terrain wavelength, 50 m reservoir) on a 2 m mesh: the
    5120 x 5120 domain size of the scaling runs of Section 6.3, whose terrain
    and physics the paper does not give."""
    rng = np.random.default_rng(seed)
    d = 10240.0 / nx if nx == ny else 2.0
    z, x, y, xc = _valley(rng, nx, ny, d, 0.2, 0.003, 3.0, 1280.0)
    rows = np.arange(ny)[:, None]
    dam = int(round(dam_row * ny / 5120))
    h = np.where(rows < dam, np.maximum(50.0 - z, 0.0), 0.0)
    zero = np.zeros((ny, nx))
    return Workload("valley_5120", nx, ny, d, d, z=z, h=np.ascontiguousarray(h),
                    qx=zero.copy(), qy=zero.copy(),
                    bc=(WALL, WALL, WALL, OUTFLOW), fric_law=FRIC_MANNING,
                    fric_coef=0.033, nsteps=20000)


def hillslope_8192(nx: int = 8192, ny: int = 8192, seed: int = 3) -> Workload:
    rng = np.random.default_rng(seed)
    d = 1.0
    Lx = nx * d
    x = _centres(nx, d)[None, :]
    z = 0.02 * (Lx - x) + 0.3 * fbm(rng, nx, ny, d, d, 64.0)
    zero = np.zeros((ny, nx))
    return Workload("hillslope_8192", nx, ny, d, d, z=np.ascontiguousarray(z),
                    h=zero.copy(), qx=zero.copy(), qy=zero.copy(),
                    bc=(WALL, OUTFLOW, WALL, WALL), fric_law=FRIC_DARCY,
                    fric_coef=0.3, rain=50.0 * MM_PER_HOUR, infil_on=1,
                    ks=1e-6, psi=0.1, dtheta=0.4, vinf=zero.copy(),
                    dt_max=1.0, nsteps=1000)


def ensemble_member(k: int, n: Optional[int] = None,
                    nmin: int = 64, nmax: int = 1024) -> Workload:
    rng = np.random.default_rng(4000 + k)
    size = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    if n is not None:
        size = n
    d = 2.0
    slope = rng.uniform(0.005, 0.05)
    rain = rng.uniform(10.0, 100.0) * MM_PER_HOUR
    manning = rng.uniform(0.02, 0.06)
    Lx = size * d
    x = _centres(size, d)[None, :]
    z = slope * (Lx - x) + 1.0 * fbm(rng, size, size, d, d,
                                     min(256.0, 0.25 * Lx))
    zero = np.zeros((size, size))
    return Workload(f"ensemble_{k}", size, size, d, d, z=np.ascontiguousarray(z),
                    h=zero.copy(), qx=zero.copy(), qy=zero.copy(),
                    bc=(WALL, OUTFLOW, WALL, WALL), fric_law=FRIC_MANNING,
                    fric_coef=manning, rain=rain, dt_max=1.0, nsteps=500)


def ensemble(count: int = 256, nmin: int = 64, nmax: int = 1024):
    return [ensemble_member(k, nmin=nmin, nmax=nmax) for k in range(count)]


def smooth_field(rng: np.random.Generator, nx: int, ny: int,
                 sigma_cells: float) -> np.ndarray:
    """Gaussian-filtered white noise scaled to max|.| = 1."""
    from scipy.ndimage import gaussian_filter
    w = rng.standard_normal((ny, nx))
    s = gaussian_filter(w, sigma_cells, mode="wrap")
    return s / np.abs(s).max()


def calibration_1024(nx: int = 1024, ny: int = 1024, seed: int = 5,
                     dam_row: int = 150, ngauges: int = 64,
                     sigma_cells: float = 20.0) -> Workload:
    rng = np.random.default_rng(seed)
    d = 2.0
    z, x, y, xc = _valley(rng, nx, ny, d, 0.2, 0.003, 3.0, 1280.0 * nx / 2048)
    rows = np.arange(ny)[:, None]
    h = np.where(rows < dam_row, np.maximum(50.0 - z, 0.0), 0.0)
    xi = smooth_field(rng, nx, ny, sigma_cells)
    fric = 0.03 * (1.0 + 0.2 * xi)
    xi_obs = smooth_field(np.random.default_rng(seed + 1000), nx, ny, sigma_cells)
    fric_obs = 0.03 * (1.0 + 0.2 * xi_obs)
    jj, ii = np.nonzero((np.abs(x - xc) <= 40.0) &
                        (rows >= dam_row) & (rows <= min(600, ny - 1)))
    cand = jj * nx + ii
    pick = rng.choice(cand.size, size=min(ngauges, cand.size), replace=False)
    gauges = np.sort(cand[pick]).astype(np.int32)
    zero = np.zeros((ny, nx))
    return Workload("calibration_1024", nx, ny, d, d, z=z,
                    h=np.ascontiguousarray(h), qx=zero.copy(), qy=zero.copy(),
                    bc=(WALL, WALL, WALL, OUTFLOW), fric_law=FRIC_MANNING,
                    fric_coef=0.03, fric=np.ascontiguousarray(fric),
                    nsteps=2000, gauges=gauges,
                    extra={"fric_obs": np.ascontiguousarray(fric_obs),
                           "every": 10})


# ----------------------------------------------------------------------------
# Generic random valid states (for single-stage parity)
# ----------------------------------------------------------------------------

def random_state(nx: int, ny: int, seed: int, dry_frac: float = 0.3,
                 film_frac: float = 0.2, dx: float = 1.0, dy: float = 1.0,
                 bc=(WALL, OUTFLOW, WALL, OUTFLOW), **kw) -> Workload:
    """Rough terrain with dry patches, 1e-3 m films and moving water."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(0.0, 1.0, (ny, nx)) + 0.05 * np.arange(nx)[None, :] * dx
    h = rng.uniform(0.0, 2.0, (ny, nx))
    r = rng.uniform(0.0, 1.0, (ny, nx))
    h = np.where(r < dry_frac, 0.0, h)
    h = np.where((r >= dry_frac) & (r < dry_frac + film_frac),
                 rng.uniform(0.5e-3, 1.5e-3, (ny, nx)), h)
    u = rng.uniform(-2.0, 2.0, (ny, nx))
    v = rng.uniform(-2.0, 2.0, (ny, nx))
    qx = np.where(h > 0, h * u, 0.0)
    qy = np.where(h > 0, h * v, 0.0)
    wl = Workload(f"random_{seed}", nx, ny, dx, dy, z=z, h=h, qx=qx, qy=qy,
                  bc=tuple(bc), **kw)
    return wl


def thacker_planar(n: int = 100, L: float = 4.0, a: float = 1.0, h0: float = 0.1,
                   eta: float = 0.5) -> Workload:
    """Thacker's planar surface in a paraboloid (Thacker 1981), at t = 0: a
    basin z = h0 (r^2 / a^2 - 1) centred in an L x L walled square of n x n
    cells, frictionless, holding water under a plane surface that rotates
    with period 2 pi / omega, omega = sqrt(2 g h0) / a, and a uniform
    velocity (u, v) = eta omega (-sin, cos)(omega t).  The shoreline stays
    inside r < a (1 + eta), away from the walls.  Values at cell centres."""
    d = L / n
    c = _centres(n, d) - 0.5 * L
    X, Y = np.meshgrid(c, c)
    z = h0 * ((X * X + Y * Y) / (a * a) - 1.0)
    omega = math.sqrt(2.0 * 9.81 * h0) / a
    surf = eta * h0 / (a * a) * (2.0 * X - eta)
    h = np.maximum(surf - z, 0.0)
    return Workload(f"thacker_{n}", n, n, d, d, z=np.ascontiguousarray(z),
                    h=np.ascontiguousarray(h), qx=np.zeros((n, n)),
                    qy=np.ascontiguousarray(h * (eta * omega)),
                    bc=(WALL, WALL, WALL, WALL), t_end=2.0 * math.pi / omega,
                    nsteps=10 ** 7)


def longest_rows(nx: int = 1 << 28, ny: int = 2) -> Workload:
    """Rows of the greatest length the library takes (2^28 cells along x,
    two rows): a sawtooth bed (0.1 mm per cell over 4096-cell teeth) under 1 m
    of water, 0.5 m more on every other 4096-cell run, at rest; walls west,
    south and north, free outflow east.  The time step is capped at 0.01 s
    (the CFL bound of this state is 0.065 s), so a step's dt is known
    without a pass over all cells.  No random draws."""
    i = np.arange(nx, dtype=np.int64)
    z_row = (i & 4095).astype(np.float64) * 1e-4
    h_row = 1.0 + 0.5 * ((i >> 12) & 1).astype(np.float64)
    del i
    z = np.empty((ny, nx))
    z[:] = z_row
    h = np.empty((ny, nx))
    h[:] = h_row
    return Workload("longest_rows", nx, ny, 1.0, 1.0, z=z, h=h,
                    qx=np.zeros((ny, nx)), qy=np.zeros((ny, nx)),
                    bc=(WALL, OUTFLOW, WALL, WALL), dt_max=0.01, nsteps=1)


def flowdir_dem(nx: int = 14786, ny: int = 10086, seed: int = 1307) -> np.ndarray:
    """A float32 DEM of the paper's flow-direction size (Section 5.2 gives
    only its dimensions): a ramp of 50 m across x plus uniform noise of 1 m,
    [ny][nx]."""
    rng = np.random.default_rng(seed)
    z = rng.random((ny, nx), dtype=np.float32)
    z += np.linspace(0.0, 50.0, nx, dtype=np.float32)[None, :]
    return z


WORKLOADS = {
    "dam_break_200": dam_break_200,
    "valley_2048": valley_2048,
    "valley_5120": valley_5120,
    "hillslope_8192": hillslope_8192,
    "calibration_1024": calibration_1024,
}
