// Discrete adjoint of the time step with respect to a spatial friction
// field (C ABI swe_adj_*, include/swe.h).
//
// The loss is the sum of squared gauge-depth misfits every `every` steps,
// L = sum_k sum_m (h^{k}[g_m] - obs[k/every - 1][m])^2 for k a multiple of
// every, and its gradient with respect to the per-cell friction coefficient
// is computed by reverse-mode differentiation of the exact discrete step
// (Sections 3.1-3.4 as implemented by the forward kernels) with the time
// step sequence frozen to the forward run's.  States are recomputed from
// sqrt(N)-spaced checkpoints segment by segment.
//
// Per step, reversed (U^n -> U* -> U** -> U^{n+1} = (U^n + U**)/2 + rain):
//   lambda_{U^n} = lambda/2;  lambda_{U**} = lambda/2
//   friction of stage 2 reversed cell by cell      -> lambda_{C2}, d/dU*, dL/dn
//   C2 = U* + dt Phi(U*):  lambda_{U*} += lambda_{C2} + VJP_Phi(U*, dt lambda_{C2})
//   friction of stage 1 reversed                   -> lambda_{C1}, d/dU^n, dL/dn
//   C1 = U^n + dt Phi(U^n): lambda_{U^n} += lambda_{C1} + VJP_Phi(U^n, dt lambda_{C1})
// The vector-Jacobian product of the rate Phi is computed per face: each
// face recomputes its four-cell stencil (primitives, the two MUSCL
// reconstructions, hydrostatic reconstruction, HLL, S and the centred term
// of its left cell) and yields the adjoint contributions to those four
// cells (face_contrib).  One tile kernel (adj_vjp_kernel) evaluates the
// faces of a tile and sums the contributions of every cell in the fixed
// order of gather_cell (no atomics), folding ghost cells back onto the cells
// they mirror.  face_contrib and gather_cell, run face by face over whole
// contribution planes, are the plain form of the same sums; the host tests
// check them against finite differences of the oracle.
//
// At points where the step is not differentiable the derivative follows
// one fixed rule: max(a, b) and min(a, b) pass the derivative of the
// selected argument (the first one on a tie), minmod passes that of the
// selected difference (none when it returns 0 for opposite signs), and the
// square root and cube root have derivative 0 at 0.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "swe.h"
#include "swe_device.h"
#include "swe_host.h"

using namespace swe_dev;
using namespace swe_host;

namespace {

constexpr int T1 = 256;  // threads of the per-cell and per-face kernels

// ---------------------------------------------------------------------------
// Reverse of the building blocks
// ---------------------------------------------------------------------------

// minmod(a, b) as the three-case definition of Section 3.4: which argument
// is returned (1 = a, 2 = b, 0 = the constant 0).
__host__ __device__ __forceinline__ int minmod_sel(double a, double b) {
    if (a >= 0.0 && b >= 0.0) return (b < a) ? 2 : 1;
    if (a <= 0.0 && b <= 0.0) return (a < b) ? 2 : 1;
    return 0;
}

__host__ __device__ __forceinline__ double sel_val(int s, double a, double b) {
    return s == 1 ? a : (s == 2 ? b : 0.0);
}

struct PrimBar {
    double h, un, ut, eta;
};

struct RecBar {
    double h_m, h_p, z_m, z_p, un_m, un_p, ut_m, ut_p;
};

__host__ __device__ __forceinline__ void zero(PrimBar& p) { p.h = p.un = p.ut = p.eta = 0.0; }
__host__ __device__ __forceinline__ void zero(RecBar& r) {
    r.h_m = r.h_p = r.z_m = r.z_p = r.un_m = r.un_p = r.ut_m = r.ut_p = 0.0;
}

// d(minmod(x, y)) routed back to s_c - s_a = x and s_b - s_c = y.  Written
// without branches: a conditional update of one of three references becomes
// a select between their addresses, which keeps the adjoints in scratch
// memory.  Adding an exact zero to the slots not selected changes no value
// (at most the sign of a zero).
__host__ __device__ __forceinline__ void route_minmod(int sel, double bar, double& abar, double& cbar,
                                             double& bbar) {
    const double x = sel == 1 ? bar : 0.0;  // through s_c - s_a
    const double y = sel == 2 ? bar : 0.0;  // through s_b - s_c
    cbar += x - y;
    abar -= x;
    bbar += y;
}

// Reverse of muscl(a, c, b): adds the adjoints of the three primitive
// vectors given the adjoint R of the reconstruction.
__host__ __device__ __forceinline__ void muscl_rev(const Prim& a, const Prim& c, const Prim& b,
                                          double h_eps, const RecBar& R, PrimBar& ab,
                                          PrimBar& cb, PrimBar& bb) {
    // forward recomputation of the selections and the values used
    double xh = c.h - a.h, yh = b.h - c.h;
    int sh = minmod_sel(xh, yh);
    double dh = sel_val(sh, xh, yh);
    double h_m = c.h - 0.5 * dh, h_p = c.h + 0.5 * dh;
    int se = minmod_sel(c.eta - a.eta, b.eta - c.eta);
    double xu = c.un - a.un, yu = b.un - c.un;
    int su = minmod_sel(xu, yu);
    double dun = sel_val(su, xu, yu);
    double xt = c.ut - a.ut, yt = b.ut - c.ut;
    int st = minmod_sel(xt, yt);
    double dut = sel_val(st, xt, yt);

    double bh_m = R.h_m, bh_p = R.h_p;
    // velocities
    cb.un += R.un_m + R.un_p;
    cb.ut += R.ut_m + R.ut_p;
    if (c.h > h_eps) {
        // one reciprocal for the six quotients by h (the branches above are
        // decided on the exact forward values; these are only arithmetic)
        const double inv = 1.0 / c.h;
        double wp = h_p * inv, wm = h_m * inv;
        double bwp = -(R.un_m * (0.5 * dun) + R.ut_m * (0.5 * dut));
        double bwm = R.un_p * (0.5 * dun) + R.ut_p * (0.5 * dut);
        double bdun = 0.5 * (wm * R.un_p - wp * R.un_m);
        double bdut = 0.5 * (wm * R.ut_p - wp * R.ut_m);
        bh_p += bwp * inv;
        cb.h -= bwp * wp * inv;
        bh_m += bwm * inv;
        cb.h -= bwm * wm * inv;
        route_minmod(su, bdun, ab.un, cb.un, bb.un);
        route_minmod(st, bdut, ab.ut, cb.ut, bb.ut);
    }
    // z = eta - h at each face
    double beta_m = R.z_m, beta_p = R.z_p;
    bh_m -= R.z_m;
    bh_p -= R.z_p;
    cb.eta += beta_m + beta_p;
    route_minmod(se, 0.5 * (beta_p - beta_m), ab.eta, cb.eta, bb.eta);
    cb.h += bh_m + bh_p;
    route_minmod(sh, 0.5 * (bh_p - bh_m), ab.h, cb.h, bb.h);
}

// Reverse of prim_x: adjoints of (h, qx, qy) of the cell as loaded (x view:
// un = u, ut = v).
__host__ __device__ __forceinline__ void prim_rev(const RawCell& r, double h_eps, const PrimBar& pb,
                                         double& bh, double& bqx, double& bqy) {
    bh = pb.h + pb.eta;  // h enters as itself and through eta = h + z
    bqx = 0.0;
    bqy = 0.0;
    if (r.h > h_eps) {
        const double inv = 1.0 / r.h;  // one reciprocal for the five quotients
        double u = r.qx * inv, v = r.qy * inv;
        bqx = pb.un * inv;
        bqy = pb.ut * inv;
        bh -= (pb.un * u + pb.ut * v) * inv;
    }
}

// Reverse of kinetic_half (one side of the kinetic flux): given the bars of
// its two moments, adds those of the side's depth and normal velocity.  The
// clamps of the support's ends at 0 take the derivative of the end itself
// when it is kept (ties included, as the first argument of max/min).
template <bool LEFT>
__host__ __device__ __forceinline__ void kinetic_half_rev(double g, double h, double un,
                                                          double bm0, double bm1, double& bh,
                                                          double& bun) {
    if (!(h > 0.0)) return;
    const double g15 = 1.5 * g;
    const double s = sqrt(g15 * h);
    const double a0 = un - s, b0 = un + s;
    const bool keep_a = LEFT ? !(a0 < 0.0) : !(0.0 < a0);
    const bool keep_b = LEFT ? !(b0 < 0.0) : !(0.0 < b0);
    const double a = keep_a ? a0 : 0.0, b = keep_b ? b0 : 0.0;
    const double w2 = b * b - a * a, w3 = b * b * b - a * a * a;
    const double i4 = 1.0 / (4.0 * s), i6 = 1.0 / (6.0 * s);
    // m0 = h w2 / (4 s), m1 = h w3 / (6 s)
    const double bw2 = bm0 * h * i4, bw3 = bm1 * h * i6;
    double bs = -(bm0 * h * w2 * i4 + bm1 * h * w3 * i6) / s;
    const double ba = -2.0 * a * bw2 - 3.0 * a * a * bw3;
    const double bb = 2.0 * b * bw2 + 3.0 * b * b * bw3;
    if (keep_a) { bun += ba; bs -= ba; }
    if (keep_b) { bun += bb; bs += bb; }
    // s = sqrt(3 g h / 2)
    bh += bm0 * w2 * i4 + bm1 * w3 * i6 + bs * g15 / (2.0 * s);
}

// Reverse of face(): adjoints of the eight inputs given those of
// (F0, F1, F2, s_L, s_R).
struct FaceBar {
    double hm, zm, unm, utm, hp, zp, unp, utp;
};

template <int FLUX = 0>
__host__ __device__ __forceinline__ FaceBar face_rev(double g, double hm, double zm, double unm,
                                            double utm, double hp, double zp, double unp,
                                            double utp, double bF0, double bF1, double bF2,
                                            double bsL, double bsR) {
    const double hg = 0.5 * g;
    // forward
    bool zs_b = zm < zp;
    double zs = zs_b ? zp : zm;
    double a1 = hm + zm - zs, a2 = hp + zp - zs;
    bool l0 = a1 < 0.0, r0 = a2 < 0.0;
    double hL = l0 ? 0.0 : a1, hR = r0 ? 0.0 : a2;
    double cL = sqrt(g * hL), cR = sqrt(g * hR);
    double l1 = unm - cL, l2 = unp - cR;
    bool c1_b = l2 < l1;
    double c1 = c1_b ? l2 : l1;
    double u1 = unm + cL, u2 = unp + cR;
    bool c2_b = u1 < u2;
    double c2 = c2_b ? u2 : u1;
    double qL = hL * unm, qR = hR * unp;
    double FL[3] = {qL, qL * unm + hg * hL * hL, qL * utm};
    double FR[3] = {qR, qR * unp + hg * hR * hR, qR * utp};
    double UL[3] = {hL, qL, hL * utm};
    double UR[3] = {hR, qR, hR * utp};
    // reverse
    FaceBar o;
    o.hm = bsL * hg * 2.0 * hm;
    o.hp = bsR * hg * 2.0 * hp;
    o.zm = o.zp = 0.0;
    o.unm = o.utm = o.unp = o.utp = 0.0;
    double bhL = -bsL * hg * 2.0 * hL;
    double bhR = -bsR * hg * 2.0 * hR;
    double bF[3] = {bF0, bF1, bF2};
    double bFL[3] = {0.0, 0.0, 0.0}, bFR[3] = {0.0, 0.0, 0.0};
    double bUL[3] = {0.0, 0.0, 0.0}, bUR[3] = {0.0, 0.0, 0.0};
    double bc1 = 0.0, bc2 = 0.0;
    double bcL = 0.0, bcR = 0.0;
    if constexpr (FLUX == 2) {
        // kinetic: F0 = m0L + m0R, F1 = m1L + m1R, F2 = m0L utm + m0R utp
        double m0L, m1L, m0R, m1R;
        kinetic_half<true>(g, hL, unm, m0L, m1L);
        kinetic_half<false>(g, hR, unp, m0R, m1R);
        o.utm += bF[2] * m0L;
        o.utp += bF[2] * m0R;
        kinetic_half_rev<true>(g, hL, unm, bF[0] + bF[2] * utm, bF[1], bhL, o.unm);
        kinetic_half_rev<false>(g, hR, unp, bF[0] + bF[2] * utp, bF[1], bhR, o.unp);
    } else if constexpr (FLUX == 1) {
        // Rusanov: F = (F(U_L) + F(U_R))/2 - c/2 (U_R - U_L),
        // c = max(|unm| + cL, |unp| + cR) (the first on ties; |x| takes the
        // derivative sign(x), +1 at 0)
        const double aL = fabs(unm) + cL, aR = fabs(unp) + cR;
        const bool right = aL < aR;
        const double c = right ? aR : aL;
        double bc = 0.0;
        for (int k = 0; k < 3; ++k) {
            bFL[k] = 0.5 * bF[k];
            bFR[k] = 0.5 * bF[k];
            bUR[k] = -0.5 * c * bF[k];
            bUL[k] = 0.5 * c * bF[k];
            bc -= 0.5 * bF[k] * (UR[k] - UL[k]);
        }
        if (right) {
            o.unp += unp < 0.0 ? -bc : bc;
            bcR += bc;
        } else {
            o.unm += unm < 0.0 ? -bc : bc;
            bcL += bc;
        }
    } else if (0.0 <= c1) {
        for (int k = 0; k < 3; ++k) bFL[k] = bF[k];
    } else if (c2 <= 0.0) {
        for (int k = 0; k < 3; ++k) bFR[k] = bF[k];
    } else {
        // one reciprocal of D = c2 - c1 > 0 for every quotient of the branch
        const double iD = 1.0 / (c2 - c1);
        const double iD2 = iD * iD;
        const double W = c1 * c2 * iD;
        const double c2D = c2 * iD, c1D = c1 * iD, c12D2 = c1 * c2 * iD2;
        for (int k = 0; k < 3; ++k) {
            double A = c2 * FL[k] - c1 * FR[k];
            double dU = UR[k] - UL[k];
            bFL[k] = bF[k] * c2D;
            bFR[k] = -bF[k] * c1D;
            bUR[k] = bF[k] * W;
            bUL[k] = -bF[k] * W;
            bc2 += bF[k] * (FL[k] * iD - A * iD2 + (c1D - c12D2) * dU);
            bc1 += bF[k] * (-FR[k] * iD + A * iD2 + (c2D + c12D2) * dU);
        }
    }
    double bqL = 0.0, bqR = 0.0;
    // U_L = (hL, qL, hL utm), U_R likewise
    bhL += bUL[0];
    bqL += bUL[1];
    bhL += bUL[2] * utm;
    o.utm += bUL[2] * hL;
    bhR += bUR[0];
    bqR += bUR[1];
    bhR += bUR[2] * utp;
    o.utp += bUR[2] * hR;
    // F(U_L) = (qL, qL unm + hg hL^2, qL utm)
    bqL += bFL[0] + bFL[1] * unm + bFL[2] * utm;
    o.unm += bFL[1] * qL;
    bhL += bFL[1] * hg * 2.0 * hL;
    o.utm += bFL[2] * qL;
    bqR += bFR[0] + bFR[1] * unp + bFR[2] * utp;
    o.unp += bFR[1] * qR;
    bhR += bFR[1] * hg * 2.0 * hR;
    o.utp += bFR[2] * qR;
    // qL = hL unm, qR = hR unp
    bhL += bqL * unm;
    o.unm += bqL * hL;
    bhR += bqR * unp;
    o.unp += bqR * hR;
    // c1 = min(unm - cL, unp - cR), c2 = max(unm + cL, unp + cR) (HLL)
    if (c1_b) { o.unp += bc1; bcR -= bc1; } else { o.unm += bc1; bcL -= bc1; }
    if (c2_b) { o.unp += bc2; bcR += bc2; } else { o.unm += bc2; bcL += bc2; }
    if (cL > 0.0) bhL += bcL * g / (2.0 * cL);
    if (cR > 0.0) bhR += bcR * g / (2.0 * cR);
    // hydrostatic reconstruction
    double bzs = 0.0;
    if (!l0) { o.hm += bhL; o.zm += bhL; bzs -= bhL; }
    if (!r0) { o.hp += bhR; o.zp += bhR; bzs -= bhR; }
    if (zs_b) o.zp += bzs; else o.zm += bzs;
    return o;
}

// Reverse of the centred source of a cell (Section 3.1).
__host__ __device__ __forceinline__ void centred_rev(double g, const Rec& r, double bfc, RecBar& R) {
    double a = (-g) * 0.5 * (r.z_p - r.z_m);
    R.h_m += bfc * a;
    R.h_p += bfc * a;
    double b = (-g) * (0.5 * (r.h_m + r.h_p));
    R.z_p += bfc * b;
    R.z_m -= bfc * b;
}

// Reverse of friction(): (h0, q0) stage input, (h1, q1) convective output.
// Given the adjoints of the outputs (bh, bq), returns those of the
// convective output (bh1, bq1), of the stage input through the friction
// factor (bh0, bq0) and of the coefficient.
__host__ __device__ __forceinline__ void friction_rev(const KParams& p, double coef, double h0,
                                             double qx0, double qy0, double h1, double qx1,
                                             double qy1, double dt, double bh, double bqx,
                                             double bqy, double& bh1, double& bqx1,
                                             double& bqy1, double& bh0, double& bqx0,
                                             double& bqy0, double& bcoef) {
    bh1 = bh;
    bh0 = bqx0 = bqy0 = bcoef = 0.0;
    if (h1 <= p.h_eps) {
        bqx1 = bqy1 = 0.0;
        return;
    }
    if (p.law == SWE_FRIC_NONE || !(h0 > p.h_eps)) {
        bqx1 = bqx;
        bqy1 = bqy;
        return;
    }
    double qn = sqrt(qx0 * qx0 + qy0 * qy0);
    double T, dT_dqn, dT_dcoef, dT_dh1;
    if (p.law == SWE_FRIC_DARCY) {
        double base = dt * qn / (h0 * h1);
        T = base * (coef / 8.0);
        dT_dcoef = base / 8.0;
        dT_dqn = dt * (coef / 8.0) / (h0 * h1);
        dT_dh1 = -T / h1;
    } else {
        double h43 = h1 * cbrt(h1);
        double base = dt * p.g * qn / (h0 * h43);
        T = base * coef * coef;
        dT_dcoef = 2.0 * base * coef;
        dT_dqn = dt * p.g * coef * coef / (h0 * h43);
        dT_dh1 = -T * (4.0 / 3.0) / h1;
    }
    double den = 1.0 + T;
    double oqx = qx1 / den, oqy = qy1 / den;
    bqx1 = bqx / den;
    bqy1 = bqy / den;
    double bden = -(bqx * oqx + bqy * oqy) / den;
    bcoef = bden * dT_dcoef;
    bh0 = -bden * T / h0;
    bh1 += bden * dT_dh1;
    double bqn = bden * dT_dqn;
    if (qn > 0.0) {
        bqx0 = bqn * qx0 / qn;
        bqy0 = bqn * qy0 / qn;
    }
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

struct AdjArgs {
    KParams p;
    const double* z;
    const double* fric;
};

// one-wave tiles for the VJP kernel, about 4096 of them, 4 to 32 rows each:
// at 1024^2 the reverse ran fastest with 4-row tiles (18 x 256 tiles; the
// halo rows of the y march cost less than the latency fewer waves leave
// exposed: 8, 2 and 1 rows were 3%, 10% and 33% slower)
constexpr int VJP_TX = 64;
inline int vjp_rows(int nx, int ny) {
    long long strips = (nx + VJP_TX - 7) / (VJP_TX - 6);
    long long ty = strips * (long long)ny / 4096;
    if (ty > 32) ty = 32;
    if (ty < 4) ty = 4;
    while ((ny + ty - 1) / ty > 65535) ty *= 2;
    return (int)ty;
}

__host__ __device__ __forceinline__ RawCell load_raw(const double* h, const double* qx,
                                            const double* qy, const double* z, int nx,
                                            int rs, int cs, double sx, double sy) {
    size_t idx = (size_t)rs * nx + cs;
    RawCell r;
    r.h = h[idx];
    r.qx = sx * qx[idx];
    r.qy = sy * qy[idx];
    r.z = z[idx];
    return r;
}

// Adjoint contributions of one face from the four cells of its stencil.
// r[k], sgn[k]: the cell at position f-2+k along the sweep (a ghost position
// holds the cell it mirrors, its discharge normal to the boundary multiplied
// by sgn[k]); muL / muR: the adjoint seeds (h, qx, qy) of the cells left of
// and right of the face, used when L_real / R_real.  out[3k + c] is the
// contribution to component c (h, qx, qy) of the cell at position f-2+k
// (ghost positions carry it to the cell they mirror, sign included): the
// face itself and the centred source of its lower/left cell.
template <int DIR, int FLUX = 0>
__host__ __device__ __forceinline__ void face_contrib_cells(const KParams& p, const RawCell r[4],
                                                            const double sgn[4], bool L_real,
                                                            bool R_real, const double muL[3],
                                                            const double muR[3],
                                                            double out[12]) {
    const double d = DIR == 0 ? p.dx : p.dy;
    Prim pr[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        pr[k] = DIR == 0 ? prim_x(r[k], p.h_eps) : to_y(prim_x(r[k], p.h_eps));
    Rec RL = muscl(pr[0], pr[1], pr[2], p.h_eps);  // cell f-1
    Rec RR = muscl(pr[1], pr[2], pr[3], p.h_eps);  // cell f

    // adjoint seeds: X_i enters Phi_i as -X_i/d
    double bL[3] = {0.0, 0.0, 0.0}, bR[3] = {0.0, 0.0, 0.0};  // (mass, normal, tangential)
    if (L_real) {
        bL[0] = -muL[0] / d;
        bL[1] = -(DIR == 0 ? muL[1] : muL[2]) / d;
        bL[2] = -(DIR == 0 ? muL[2] : muL[1]) / d;
    }
    if (R_real) {
        bR[0] = -muR[0] / d;
        bR[1] = -(DIR == 0 ? muR[1] : muR[2]) / d;
        bR[2] = -(DIR == 0 ? muR[2] : muR[1]) / d;
    }
    FaceBar fb = face_rev<FLUX>(p.g, RL.h_p, RL.z_p, RL.un_p, RL.ut_p, RR.h_m, RR.z_m,
                                RR.un_m, RR.ut_m, bL[0] - bR[0], bL[1] - bR[1], bL[2] - bR[2],
                                bL[1], -bR[1]);
    RecBar RLb, RRb;
    zero(RLb);
    zero(RRb);
    RLb.h_p = fb.hm;
    RLb.z_p = fb.zm;
    RLb.un_p = fb.unm;
    RLb.ut_p = fb.utm;
    RRb.h_m = fb.hp;
    RRb.z_m = fb.zp;
    RRb.un_m = fb.unp;
    RRb.ut_m = fb.utp;
    // centred source of the left cell: X1 = ... - fc
    if (L_real) centred_rev(p.g, RL, -bL[1], RLb);
    PrimBar pb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) zero(pb[k]);
    muscl_rev(pr[0], pr[1], pr[2], p.h_eps, RLb, pb[0], pb[1], pb[2]);
    muscl_rev(pr[1], pr[2], pr[3], p.h_eps, RRb, pb[1], pb[2], pb[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        PrimBar xb = pb[k];
        if (DIR == 1) {  // back to the x view of the primitives
            double t = xb.un;
            xb.un = xb.ut;
            xb.ut = t;
        }
        double bh, bqx, bqy;
        prim_rev(r[k], p.h_eps, xb, bh, bqx, bqy);
        // the ghost's discharge is sign * source discharge
        if (DIR == 0) bqx *= sgn[k]; else bqy *= sgn[k];
        out[3 * k + 0] = bh;
        out[3 * k + 1] = bqx;
        out[3 * k + 2] = bqy;
    }
}

// The same, loading the stencil: DIR 0: x-face f of row `line` (between
// columns f-1 and f, f = 0..nx); DIR 1: y-face f of column `line` (between
// rows f-1 and f, f = 0..ny).
template <int DIR, int FLUX = 0>
__host__ __device__ __forceinline__ void face_contrib(const KParams& p, const double* z,
                                                      const double* h, const double* qx,
                                                      const double* qy, const double* mu_h,
                                                      const double* mu_qx, const double* mu_qy,
                                                      int f, int line, double out[12]) {
    const int nx = p.nx, ny = p.ny;
    const int n_along = DIR == 0 ? nx : ny;
    RawCell r[4];
    double sgn[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int pos = f - 2 + k;
        double sg;
        if (DIR == 0) {
            int cs = map_index(pos, nx, p.bcw, p.bce, sg);
            r[k] = load_raw(h, qx, qy, z, nx, line, cs, sg, 1.0);
        } else {
            int rs = map_index(pos, ny, p.bcs, p.bcn, sg);
            r[k] = load_raw(h, qx, qy, z, nx, rs, line, 1.0, sg);
        }
        sgn[k] = sg;
    }
    const bool L_real = f - 1 >= 0 && f - 1 < n_along;
    const bool R_real = f < n_along;
    double muL[3] = {0.0, 0.0, 0.0}, muR[3] = {0.0, 0.0, 0.0};
    if (L_real) {
        size_t idx = DIR == 0 ? (size_t)line * nx + (f - 1) : (size_t)(f - 1) * nx + line;
        muL[0] = mu_h[idx];
        muL[1] = mu_qx[idx];
        muL[2] = mu_qy[idx];
    }
    if (R_real) {
        size_t idx = DIR == 0 ? (size_t)line * nx + f : (size_t)f * nx + line;
        muR[0] = mu_h[idx];
        muR[1] = mu_qx[idx];
        muR[2] = mu_qy[idx];
    }
    face_contrib_cells<DIR, FLUX>(p, r, sgn, L_real, R_real, muL, muR, out);
}

// The face contributions addressed to cell (i, j), summed in a fixed order:
// interior positions, then the ghost positions that mirror it; xc and yc
// hold 12 planes (slot 0..3 x component) of the x-faces (ny x (nx+1)) and
// the y-faces ((ny+1) x nx).
__host__ __device__ __forceinline__ void add_contrib(const double* buf, size_t plane, size_t fidx,
                                            int slot, double& h, double& qx, double& qy) {
    h += buf[(size_t)(3 * slot + 0) * plane + fidx];
    qx += buf[(size_t)(3 * slot + 1) * plane + fidx];
    qy += buf[(size_t)(3 * slot + 2) * plane + fidx];
}

__host__ __device__ __forceinline__ void gather_cell(const KParams& p, const double* xc,
                                                     const double* yc, int i, int j,
                                                     double& sh, double& sqx, double& sqy) {
    const int nx = p.nx, ny = p.ny;
    sh = sqx = sqy = 0.0;
    // x-faces of row j: faces f with i in [f-2, f+1], slot i-f+2
    {
        const size_t plane = (size_t)ny * (nx + 1);
        const size_t row = (size_t)j * (nx + 1);
        for (int f = (i - 1 > 0 ? i - 1 : 0); f <= (i + 2 < nx ? i + 2 : nx); ++f)
            add_contrib(xc, plane, row + f, i - f + 2, sh, sqx, sqy);
        // ghost columns -1, -2 (west) and nx, nx+1 (east)
        if (i == 0) {
            add_contrib(xc, plane, row + 0, 1, sh, sqx, sqy);  // column -1
            add_contrib(xc, plane, row + 1, 0, sh, sqx, sqy);
            if (p.bcw == SWE_BC_OUTFLOW) add_contrib(xc, plane, row + 0, 0, sh, sqx, sqy);
        }
        if (i == 1 && p.bcw == SWE_BC_WALL) add_contrib(xc, plane, row + 0, 0, sh, sqx, sqy);
        if (i == nx - 1) {
            add_contrib(xc, plane, row + nx - 1, 3, sh, sqx, sqy);  // column nx
            add_contrib(xc, plane, row + nx, 2, sh, sqx, sqy);
            if (p.bce == SWE_BC_OUTFLOW) add_contrib(xc, plane, row + nx, 3, sh, sqx, sqy);
        }
        if (i == nx - 2 && p.bce == SWE_BC_WALL)
            add_contrib(xc, plane, row + nx, 3, sh, sqx, sqy);
    }
    // y-faces of column i: faces f with j in [f-2, f+1]
    {
        const size_t plane = (size_t)(ny + 1) * nx;
        for (int f = (j - 1 > 0 ? j - 1 : 0); f <= (j + 2 < ny ? j + 2 : ny); ++f)
            add_contrib(yc, plane, (size_t)f * nx + i, j - f + 2, sh, sqx, sqy);
        if (j == 0) {
            add_contrib(yc, plane, (size_t)0 * nx + i, 1, sh, sqx, sqy);  // row -1
            add_contrib(yc, plane, (size_t)1 * nx + i, 0, sh, sqx, sqy);
            if (p.bcs == SWE_BC_OUTFLOW) add_contrib(yc, plane, (size_t)0 * nx + i, 0, sh, sqx, sqy);
        }
        if (j == 1 && p.bcs == SWE_BC_WALL) add_contrib(yc, plane, (size_t)0 * nx + i, 0, sh, sqx, sqy);
        if (j == ny - 1) {
            add_contrib(yc, plane, (size_t)(ny - 1) * nx + i, 3, sh, sqx, sqy);  // row ny
            add_contrib(yc, plane, (size_t)ny * nx + i, 2, sh, sqx, sqy);
            if (p.bcn == SWE_BC_OUTFLOW) add_contrib(yc, plane, (size_t)ny * nx + i, 3, sh, sqx, sqy);
        }
        if (j == ny - 2 && p.bcn == SWE_BC_WALL)
            add_contrib(yc, plane, (size_t)ny * nx + i, 3, sh, sqx, sqy);
    }
}

// VJP of Phi over one tile (64 lanes = columns, rows y0 .. y1-1), cell by
// cell: the bars of each face (face_rev: the hydrostatic reconstruction and
// the flux reversed) go to the reconstructions of its two cells; each
// cell's reconstruction is reversed once (muscl_rev) with the bars of both
// its faces and of its centred source; the resulting bars of the
// primitives are summed per cell (from the reconstructions of the cell and
// of its two neighbours) and reversed once (prim_rev).  Ghost positions
// (-2, -1, n, n+1 along a sweep) carry their bars to the cells they mirror,
// discharge sign included.  lambda += x part + y part.
//
// x: lane t owns column c = strip * (64 - 6) - 3 + t (outputs: lanes
// 3 .. 60); neighbours exchange by DPP lane shifts, ghost columns fold by
// lane shuffles.  y: down the column, iteration n loads row n, forms the
// reconstruction of row n-1, reverses face n-1 (between rows n-2 and n-1)
// and the reconstruction of row n-2, and completes row n-3, which no later
// reconstruction touches.  Faces with no real cell on either side get zero
// seeds, so their bars are exactly zero.
template <int TXT, int FLUX>
__global__ __launch_bounds__(TXT) void adj_vjp_kernel(AdjArgs a, const double* __restrict__ h,
                                                      const double* __restrict__ qx,
                                                      const double* __restrict__ qy,
                                                      const double* __restrict__ mu_h,
                                                      const double* __restrict__ mu_qx,
                                                      const double* __restrict__ mu_qy,
                                                      double* __restrict__ lh,
                                                      double* __restrict__ lqx,
                                                      double* __restrict__ lqy, int ty) {
    static_assert(TXT == 64, "one wave per tile: neighbours move by DPP lane shifts");
    constexpr int H = 3, OUTW = TXT - 2 * H;
    const KParams& p = a.p;
    const int nx = p.nx, ny = p.ny;
    const int t = threadIdx.x;
    const int c = (int)blockIdx.x * OUTW - H + t;
    const int y0 = (int)blockIdx.y * ty;
    const int y1 = y0 + ty < ny ? y0 + ty : ny;
    double sx;
    const int cs = map_index(c, nx, p.bcw, p.bce, sx);
    const bool col_real = c >= 0 && c < nx;
    const bool out = t >= H && t < TXT - H && col_real;
    // byte offsets within a row (see at()): the mapped column, the seeds'
    // column (0 off the grid, where the seed is 0) and the output column
    uint32_t os = (uint32_t)cs * (uint32_t)sizeof(double);
    uint32_t om = (uint32_t)(col_real ? c : 0) * (uint32_t)sizeof(double);
    uint32_t oc = (uint32_t)c * (uint32_t)sizeof(double);
    // v / dx and v / dy: products when both are powers of two (equal to the
    // quotients bit for bit)
    auto over_dx = [&](double v) { return p.dxy_pow2 ? v * p.inv_dx : v / p.dx; };
    auto over_dy = [&](double v) { return p.dxy_pow2 ? v * p.inv_dy : v / p.dy; };

    // lanes whose ghost columns fold into this column: west (w1, w2) and
    // east (e1, e2); a lane with none reads itself with weight 0
    const bool wall_w = p.bcw == SWE_BC_WALL, wall_e = p.bce == SWE_BC_WALL;
    int w1 = t, w2 = t, e1 = t, e2 = t;
    double kw1 = 0.0, kw2 = 0.0, ke1 = 0.0, ke2 = 0.0;
    if (c == 0) { w1 = t - 1; kw1 = 1.0; if (!wall_w) { w2 = t - 2; kw2 = 1.0; } }
    if (c == 1 && wall_w) { w2 = t - 3; kw2 = 1.0; }
    if (c == nx - 1) { e1 = t + 1; ke1 = 1.0; if (!wall_e) { e2 = t + 2; ke2 = 1.0; } }
    if (c == nx - 2 && wall_e) { e2 = t + 3; ke2 = 1.0; }
    w1 = w1 < 0 ? 0 : w1; w2 = w2 < 0 ? 0 : w2;
    e1 = e1 > TXT - 1 ? TXT - 1 : e1; e2 = e2 > TXT - 1 ? TXT - 1 : e2;

    // row r of this column as loaded (ghost rows mapped, discharge signs
    // applied) and its seed (0 off the grid)
    auto load = [&](int r, RawCell& cell, double& sy, double m[3]) {
        const int rs = map_index(r, ny, p.bcs, p.bcn, sy);
        const size_t ro = (size_t)rs * nx;
        cell.h = at(h + ro, os);
        cell.qx = sx * at(qx + ro, os);
        cell.qy = sy * at(qy + ro, os);
        cell.z = at(a.z + ro, os);
        const bool row_real = r >= 0 && r < ny;
        const bool real = row_real && col_real;
        const size_t rm = (size_t)(row_real ? r : 0) * nx;
        m[0] = real ? at(mu_h + rm, om) : 0.0;
        m[1] = real ? at(mu_qx + rm, om) : 0.0;
        m[2] = real ? at(mu_qy + rm, om) : 0.0;
    };
    auto shl = [](const Prim& v) {
        Prim o;
        o.h = from_left(v.h); o.un = from_left(v.un); o.ut = from_left(v.ut);
        o.eta = from_left(v.eta);
        return o;
    };
    auto shr = [](const Prim& v) {
        Prim o;
        o.h = from_right(v.h); o.un = from_right(v.un); o.ut = from_right(v.ut);
        o.eta = from_right(v.eta);
        return o;
    };

    // x part of a row (all lanes; the row is the same for the whole wave)
    auto xpart = [&](const RawCell& w, const double m[3], double o[3]) {
        const Prim P = prim_x(w, p.h_eps);
        const Prim Pl = shl(P), Pr = shr(P);
        const Rec R = muscl(Pl, P, Pr, p.h_eps);
        // X_i enters Phi_i as -X_i / dx
        const double b0 = over_dx(-m[0]), b1 = over_dx(-m[1]), b2 = over_dx(-m[2]);
        const double l0 = from_left(b0), l1 = from_left(b1), l2 = from_left(b2);
        // face c, between column c-1 (lane t-1, its p side) and c
        const FaceBar fb = face_rev<FLUX>(p.g, from_left(R.h_p), from_left(R.z_p),
                                          from_left(R.un_p), from_left(R.ut_p), R.h_m, R.z_m,
                                          R.un_m, R.ut_m, l0 - b0, l1 - b1, l2 - b2, l1, -b1);
        // this cell's reconstruction: m side from face c, p side from face
        // c+1 (lane t+1), and its centred source
        RecBar rb;
        rb.h_m = fb.hp; rb.z_m = fb.zp; rb.un_m = fb.unp; rb.ut_m = fb.utp;
        rb.h_p = from_right(fb.hm); rb.z_p = from_right(fb.zm);
        rb.un_p = from_right(fb.unm); rb.ut_p = from_right(fb.utm);
        centred_rev(p.g, R, -b1, rb);
        PrimBar pa, pc, pb;
        zero(pa); zero(pc); zero(pb);
        muscl_rev(Pl, P, Pr, p.h_eps, rb, pa, pc, pb);
        // bars of this cell's primitives: from the reconstruction of the
        // left neighbour (its b), its own (c) and the right one's (a)
        PrimBar s;
        s.h = from_left(pb.h) + pc.h + from_right(pa.h);
        s.un = from_left(pb.un) + pc.un + from_right(pa.un);
        s.ut = from_left(pb.ut) + pc.ut + from_right(pa.ut);
        s.eta = from_left(pb.eta) + pc.eta + from_right(pa.eta);
        double bh, bqx, bqy;
        prim_rev(w, p.h_eps, s, bh, bqx, bqy);
        bqx *= sx;
        // ghost columns fold into the columns they mirror
        const double v[3] = {bh, bqx, bqy};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double gw1 = __shfl(v[q], w1, TXT), gw2 = __shfl(v[q], w2, TXT);
            const double ge1 = __shfl(v[q], e1, TXT), ge2 = __shfl(v[q], e2, TXT);
            o[q] = v[q] + kw1 * gw1 + kw2 * gw2 + ke1 * ge1 + ke2 * ge2;
        }
    };

    // per-lane slots (no lane reads another's): the x parts of the last
    // four rows (slot n & 3) and the y bars of the ghost rows -1 and -2
    __shared__ double Xs[4][3][TXT];
    __shared__ double Gs[2][3][TXT];

    // ---- y window (rows relative to the iteration's new row n) ----
    RawCell r3, r2, r1;                  // rows n-3, n-2, n-1 as loaded (z unused)
    Prim P3, P2, P1;                     // y-view primitives of rows n-3 .. n-1
    Rec R2;                              // reconstruction of row n-2
    RecBar M2;                           // its m-side bars (face n-2)
    double bY2[3] = {0.0, 0.0, 0.0}, bY1[3] = {0.0, 0.0, 0.0};  // seeds (y view)
    PrimBar A, B;                        // partial bars of rows n-3 and n-2
    zero(A); zero(B); zero(M2);
    R2.h_m = R2.h_p = R2.z_m = R2.z_p = R2.un_m = R2.un_p = R2.ut_m = R2.ut_p = 0.0;
    P3.h = P3.un = P3.ut = P3.eta = 0.0;
    P2 = P1 = P3;
    r3.h = r3.qx = r3.qy = r3.z = 0.0;
    r2 = r1 = r3;

    const int n_end = y1 == ny ? y1 + 4 : y1 + 2;
    for (int n = y0 - 3; n <= n_end; ++n) {
        // the offsets are opaque from here, so that each access takes its
        // row in scalar registers rather than a base folded before the loop
        asm volatile("" : "+v"(os), "+v"(om), "+v"(oc));
        RawCell r0;
        double s0, m0[3];
        load(n, r0, s0, m0);
        const Prim P0 = to_y(prim_x(r0, p.h_eps));
        const double bY0[3] = {over_dy(-m0[0]), over_dy(-m0[2]), over_dy(-m0[1])};

        // x part of row n
        if (n >= y0 && n < y1) {
            double X0[3];
            xpart(r0, m0, X0);
            Xs[n & 3][0][t] = X0[0];
            Xs[n & 3][1][t] = X0[1];
            Xs[n & 3][2][t] = X0[2];
        }

        Rec R1;
        R1.h_m = R1.h_p = R1.z_m = R1.z_p = R1.un_m = R1.un_p = R1.ut_m = R1.ut_p = 0.0;
        RecBar M1;
        zero(M1);
        PrimBar C;  // bars of row n-1 from the reconstruction of row n-2
        zero(C);
        if (n >= y0 - 1) R1 = muscl(P2, P1, P0, p.h_eps);
        if (n >= y0) {
            // face n-1, between rows n-2 (p side of R2) and n-1 (m side of R1)
            const FaceBar fb = face_rev<FLUX>(p.g, R2.h_p, R2.z_p, R2.un_p, R2.ut_p, R1.h_m,
                                              R1.z_m, R1.un_m, R1.ut_m, bY2[0] - bY1[0],
                                              bY2[1] - bY1[1], bY2[2] - bY1[2], bY2[1],
                                              -bY1[1]);
            M1.h_m = fb.hp; M1.z_m = fb.zp; M1.un_m = fb.unp; M1.ut_m = fb.utp;
            if (n >= y0 + 1) {
                // row n-2's reconstruction: m side (face n-2), p side (face
                // n-1), centred source; reversed once
                RecBar rb = M2;
                rb.h_p = fb.hm; rb.z_p = fb.zm; rb.un_p = fb.unm; rb.ut_p = fb.utm;
                centred_rev(p.g, R2, -bY2[1], rb);
                PrimBar pa, pc;
                zero(pa); zero(pc);
                muscl_rev(P3, P2, P1, p.h_eps, rb, pa, pc, C);
                A.h += pa.h; A.un += pa.un; A.ut += pa.ut; A.eta += pa.eta;
                B.h += pc.h; B.un += pc.un; B.ut += pc.ut; B.eta += pc.eta;
            }
        }

        // ---- row n-3 is complete ----
        const int jd = n - 3;
        if (n >= y0 + 1) {
            PrimBar xb;  // back to the x view of the primitives
            xb.h = A.h; xb.un = A.ut; xb.ut = A.un; xb.eta = A.eta;
            double yb[3], s3;
            prim_rev(r3, p.h_eps, xb, yb[0], yb[1], yb[2]);
            (void)map_index(jd, ny, p.bcs, p.bcn, s3);
            yb[2] *= s3;
            if (jd == -1 || jd == -2) {
#pragma unroll
                for (int q = 0; q < 3; ++q) Gs[-1 - jd][q][t] = yb[q];
            }
            if (jd >= y0 && jd < y1 && out) {
                double tot[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    tot[q] = Xs[jd & 3][q][t] + yb[q];
                    // ghost rows below fold into rows 0 and 1
                    if (jd == 0)
                        tot[q] += Gs[0][q][t] + (p.bcs != SWE_BC_WALL ? Gs[1][q][t] : 0.0);
                    if (jd == 1 && p.bcs == SWE_BC_WALL) tot[q] += Gs[1][q][t];
                }
                const size_t ro = (size_t)jd * nx;
                at(lh + ro, oc) += tot[0];
                at(lqx + ro, oc) += tot[1];
                at(lqy + ro, oc) += tot[2];
            }
            // ghost rows above fold into rows ny-1 and ny-2 (written before)
            if (out && (jd == ny || jd == ny + 1)) {
                int dst = -1;
                if (jd == ny) dst = ny - 1;
                if (jd == ny + 1) dst = p.bcn == SWE_BC_WALL ? ny - 2 : ny - 1;
                if (dst >= y0 && dst < y1) {
                    const size_t ro = (size_t)dst * nx;
                    at(lh + ro, oc) += yb[0];
                    at(lqx + ro, oc) += yb[1];
                    at(lqy + ro, oc) += yb[2];
                }
            }
        }

        // ---- shift the window ----
        r3 = r2; r2 = r1; r1 = r0;
        P3 = P2; P2 = P1; P1 = P0;
        R2 = R1;
        M2 = M1;
        A = B;
        B = C;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            bY2[q] = bY1[q];
            bY1[q] = bY0[q];
        }
    }
}

// U_out = friction(U_in + dt Phi(U_in)) cell by cell (a stage output).
__global__ __launch_bounds__(T1) void stage_out_kernel(KParams p, const double* __restrict__ fric,
                                                       const double* __restrict__ h,
                                                       const double* __restrict__ qx,
                                                       const double* __restrict__ qy,
                                                       const double* __restrict__ ph,
                                                       const double* __restrict__ pqx,
                                                       const double* __restrict__ pqy, double dt,
                                                       double* __restrict__ ho,
                                                       double* __restrict__ qxo,
                                                       double* __restrict__ qyo, size_t n) {
    size_t i = (size_t)blockIdx.x * T1 + threadIdx.x;
    if (i >= n) return;
    double h1 = h[i] + dt * ph[i];
    double qx1 = qx[i] + dt * pqx[i];
    double qy1 = qy[i] + dt * pqy[i];
    friction(p, fric ? fric[i] : p.coef, h[i], qx[i], qy[i], h1, qx1, qy1, dt);
    ho[i] = h1;
    qxo[i] = qx1;
    qyo[i] = qy1;
}

// Reverse of a stage's friction and of C = U_in + dt Phi(U_in) up to the
// rate: given the adjoint of the stage output (bo), writes
//   lam_in  = bC + (friction-factor part)           [mode 0]
//   lam_in += the same                               [mode 1]
//   lam_in  = base/2 + the same                      [mode 2: Heun's other half]
//   mu      = dt * bC                              (seed for VJP_Phi)
//   grad   += d/dcoef
// STAGE 2 also forms the Heun split: its output adjoint is half of `lam`,
// and the other half seeds lam_n.
// Stage 2 of the reverse of a step, fused with the rebuild of its input: U*
// = friction(U^k + dt Phi(U^k)) (what stage_out_kernel computes) is formed
// per cell, written to us (the VJP that follows reads it) and used as the
// stage input of the friction reversal with output adjoint lam/2, as in
// adj_stage_kernel (mode 0).  One kernel and one pass over U* fewer.
__global__ __launch_bounds__(T1) void adj_stage2_kernel(
    KParams p, const double* __restrict__ fric, const double* __restrict__ h,
    const double* __restrict__ qx, const double* __restrict__ qy,
    const double* __restrict__ ph, const double* __restrict__ pqx,
    const double* __restrict__ pqy, const double* __restrict__ ph2,
    const double* __restrict__ pqx2, const double* __restrict__ pqy2, double dt,
    const double* __restrict__ bo_h, const double* __restrict__ bo_qx,
    const double* __restrict__ bo_qy, double* __restrict__ us_h, double* __restrict__ us_qx,
    double* __restrict__ us_qy, double* __restrict__ lin_h, double* __restrict__ lin_qx,
    double* __restrict__ lin_qy, double* __restrict__ mu_h, double* __restrict__ mu_qx,
    double* __restrict__ mu_qy, double* __restrict__ grad, size_t n) {
    size_t i = (size_t)blockIdx.x * T1 + threadIdx.x;
    if (i >= n) return;
    const double coef = fric ? fric[i] : p.coef;
    // U*
    double h0 = h[i] + dt * ph[i];
    double qx0 = qx[i] + dt * pqx[i];
    double qy0 = qy[i] + dt * pqy[i];
    friction(p, coef, h[i], qx[i], qy[i], h0, qx0, qy0, dt);
    us_h[i] = h0;
    us_qx[i] = qx0;
    us_qy[i] = qy0;
    // stage 2 from U*
    double h1 = h0 + dt * ph2[i];
    double qx1 = qx0 + dt * pqx2[i];
    double qy1 = qy0 + dt * pqy2[i];
    double bh1, bqx1, bqy1, bh0, bqx0, bqy0, bc;
    friction_rev(p, coef, h0, qx0, qy0, h1, qx1, qy1, dt, 0.5 * bo_h[i], 0.5 * bo_qx[i],
                 0.5 * bo_qy[i], bh1, bqx1, bqy1, bh0, bqx0, bqy0, bc);
    lin_h[i] = bh1 + bh0;
    lin_qx[i] = bqx1 + bqx0;
    lin_qy[i] = bqy1 + bqy0;
    mu_h[i] = dt * bh1;
    mu_qx[i] = dt * bqx1;
    mu_qy[i] = dt * bqy1;
    if (grad) grad[i] += bc;
}

__global__ __launch_bounds__(T1) void adj_stage_kernel(
    KParams p, const double* __restrict__ fric, const double* __restrict__ h,
    const double* __restrict__ qx, const double* __restrict__ qy,
    const double* __restrict__ ph, const double* __restrict__ pqx,
    const double* __restrict__ pqy, double dt, const double* __restrict__ bo_h,
    const double* __restrict__ bo_qx, const double* __restrict__ bo_qy, double bo_scale,
    double* __restrict__ lin_h, double* __restrict__ lin_qx, double* __restrict__ lin_qy,
    int mode, const double* __restrict__ base_h, const double* __restrict__ base_qx,
    const double* __restrict__ base_qy, double* __restrict__ mu_h, double* __restrict__ mu_qx,
    double* __restrict__ mu_qy, double* __restrict__ grad, size_t n) {
    size_t i = (size_t)blockIdx.x * T1 + threadIdx.x;
    if (i >= n) return;
    double h0 = h[i], qx0 = qx[i], qy0 = qy[i];
    double h1 = h0 + dt * ph[i];
    double qx1 = qx0 + dt * pqx[i];
    double qy1 = qy0 + dt * pqy[i];
    double coef = fric ? fric[i] : p.coef;
    double bh1, bqx1, bqy1, bh0, bqx0, bqy0, bc;
    friction_rev(p, coef, h0, qx0, qy0, h1, qx1, qy1, dt, bo_scale * bo_h[i],
                 bo_scale * bo_qx[i], bo_scale * bo_qy[i], bh1, bqx1, bqy1, bh0, bqx0, bqy0,
                 bc);
    double lh = bh1 + bh0, lqx = bqx1 + bqx0, lqy = bqy1 + bqy0;
    if (mode == 1) {
        lin_h[i] += lh;
        lin_qx[i] += lqx;
        lin_qy[i] += lqy;
    } else if (mode == 2) {
        lin_h[i] = 0.5 * base_h[i] + lh;
        lin_qx[i] = 0.5 * base_qx[i] + lqx;
        lin_qy[i] = 0.5 * base_qy[i] + lqy;
    } else {
        lin_h[i] = lh;
        lin_qx[i] = lqx;
        lin_qy[i] = lqy;
    }
    mu_h[i] = dt * bh1;
    mu_qx[i] = dt * bqx1;
    mu_qy[i] = dt * bqy1;
    if (grad) grad[i] += bc;
}

// h at the gauges -> row of the gauge series
__global__ void gauge_kernel(const double* __restrict__ h, const int* __restrict__ gauges,
                             int ng, double* __restrict__ out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < ng) out[k] = h[gauges[k]];
}

// lambda_h[g_m] += 2 (h[g_m] - obs_m), one thread in gauge order (gauges may
// repeat)
__global__ void inject_kernel(const double* __restrict__ series, const double* __restrict__ obs,
                              const int* __restrict__ gauges, int ng, double* __restrict__ lh) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        for (int k = 0; k < ng; ++k) lh[gauges[k]] += 2.0 * (series[k] - obs[k]);
}

// loss = sum (series - obs)^2 in index order (single thread: a few
// thousand terms)
__global__ void loss_kernel(const double* __restrict__ series, const double* __restrict__ obs,
                            size_t n, double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (size_t k = 0; k < n; ++k) {
            double e = series[k] - obs[k];
            s += e * e;
        }
        *out = s;
    }
}

// Forward stages of one tile grid (the same tile routine as the
// single-simulation context).
template <int STAGE, int TXT, bool PHI2, int FLUX>
__global__ __launch_bounds__(TXT) void fwd_stage_kernel(MemberArgs m, TileIO io, int ty) {
    const int y0 = blockIdx.y * ty;
    const int y1 = min(y0 + ty, m.p.ny);
    stage_tile<STAGE, TXT, false, 2, FLUX, PHI2>(m, io, blockIdx.x, y0, y1,
                                              blockIdx.x == 0 && blockIdx.y == 0,
                                              blockIdx.x + blockIdx.y * gridDim.x);
}

// One stage over the whole grid with the default tiling of its size; PHI2:
// stage 2 also writes Phi(U*) to io.ph2/pqx2/pqy2.
template <int STAGE, bool PHI2 = false>
void launch_fwd(const swe_params& prm, hipStream_t s, const MemberArgs& m, const TileIO& io) {
    const int tx = default_tx(prm.nx, prm.ny);
    const int ty = auto_rows(prm.nx, prm.ny, tx);
    const dim3 grid(strips_of(prm.nx, tx), (prm.ny + ty - 1) / ty);
    if (prm.flux == 2) {
        if (tx == 64)
            hipLaunchKernelGGL((fwd_stage_kernel<STAGE, 64, PHI2, 2>), grid, dim3(64), 0, s, m,
                               io, ty);
        else
            hipLaunchKernelGGL((fwd_stage_kernel<STAGE, 256, PHI2, 2>), grid, dim3(256), 0, s, m,
                               io, ty);
    } else if (prm.flux == 1) {
        if (tx == 64)
            hipLaunchKernelGGL((fwd_stage_kernel<STAGE, 64, PHI2, 1>), grid, dim3(64), 0, s, m,
                               io, ty);
        else
            hipLaunchKernelGGL((fwd_stage_kernel<STAGE, 256, PHI2, 1>), grid, dim3(256), 0, s, m,
                               io, ty);
    } else if (tx == 64) {
        hipLaunchKernelGGL((fwd_stage_kernel<STAGE, 64, PHI2, 0>), grid, dim3(64), 0, s, m, io,
                           ty);
    } else {
        hipLaunchKernelGGL((fwd_stage_kernel<STAGE, 256, PHI2, 0>), grid, dim3(256), 0, s, m, io,
                           ty);
    }
}

// Per-step reset of the time bookkeeping (the status flags stay sticky).
__global__ void reset_step_kernel(DevScalars* sc) {
    if (blockIdx.x == 0 && threadIdx.x < AMAX_SPREAD) {
        sc->amax[0][threadIdx.x][0] = sc->amax[0][threadIdx.x][1] = 0ull;
        sc->amax[1][threadIdx.x][0] = sc->amax[1][threadIdx.x][1] = 0ull;
    }
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc->t[0] = sc->t[1] = 0.0;
        sc->steps[0] = sc->steps[1] = 0;
    }
}

__global__ void fill_kernel(double* __restrict__ a, double v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) a[i] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------

struct swe_adj {
    swe_params prm;
    MemberArgs m;          // forward view (state buffers re-pointed per launch)
    AdjArgs aa;
    hipStream_t stream;
    int nsteps, every, ngauges, ckpt;
    int nrows;             // loss evaluations = nsteps / every
    const int* gauges;     // device
    const double* obs;     // device, nrows x ngauges
    const double* h0;      // initial state (caller's buffers)
    const double* qx0;
    const double* qy0;
    double* dts;           // device, nsteps
    bool dts_frozen;
    double* series;        // device, nrows x ngauges
    double* ckpts;         // device, nckpt x 3N
    double* seg;           // device, (ckpt + 1) x 3N
    double* segphi;        // Phi(U^k) of the recomputed segment steps, ckpt x 3N
    double* segphi2;       // Phi(U*) of the same steps, ckpt x 3N
    bool last_kept;        // the forward pass left the last segment's states and
                           // rates in seg / segphi / segphi2
    double* ust;           // U* (3N)
    double* phi;           // Phi (3N)
    double* phi0;          // Phi(U^k) kept for the reverse of stage 1 (3N)
    double* lamA;          // lambda of U^n (3N)
    double* lamB;          // lambda of U* (3N)
    double* lam;           // lambda of U^{n+1} (3N)
    double* mu;            // VJP seed (3N)
    double* loss_dev;
    size_t n;
};

namespace {

// Byte offsets of the workspace's parts, from one place for both the size
// a caller allocates and the carve-up of swe_adj_create.  A checkpoint
// spacing beyond the step count means one segment: the whole run.
struct AdjLayout {
    int ckpt;
    size_t scalars, loss, dts, series, ckpts, seg, segphi, segphi2, tail, total;
};

AdjLayout adj_layout(const swe_params* p, int nsteps, int ckpt, int ngauges, int every) {
    AdjLayout L;
    L.ckpt = ckpt < nsteps ? ckpt : nsteps;
    size_t an = align256(ncells(p) * sizeof(double));
    size_t nck = (nsteps + L.ckpt - 1) / L.ckpt;
    size_t rows = every > 0 ? nsteps / every : 0;
    size_t o = 0;
    L.scalars = o; o += SCALAR_BYTES;
    L.loss = o; o += 256;
    L.dts = o; o += align256(nsteps * sizeof(double));
    L.series = o; o += align256(rows * (size_t)ngauges * sizeof(double));
    L.ckpts = o; o += 3 * an * nck;
    L.seg = o; o += 3 * an * (L.ckpt + 1);
    L.segphi = o; o += 3 * an * L.ckpt;
    L.segphi2 = o; o += 3 * an * L.ckpt;
    L.tail = o; o += 3 * an * 7;  // ust, phi, phi0, lamA, lamB, lam, mu
    L.total = o;
    return L;
}

size_t adj_bytes(const swe_params* p, int nsteps, int ckpt, int ngauges, int every) {
    return adj_layout(p, nsteps, ckpt, ngauges, every).total;
}

inline double* plane(double* base, size_t n, int k) { return base + (size_t)k * n; }
inline const double* plane(const double* base, size_t n, int k) { return base + (size_t)k * n; }

int blocks(size_t n) { return (int)((n + T1 - 1) / T1); }

// One forward step U_in -> U_out with a frozen dt (dt_fixed > 0) or the CFL
// dt (dt_fixed = 0, logged to dts[k]).  phi_out and phi2_out (optional)
// receive Phi(U_in) and Phi(U*), which the two stages compute anyway.
void fwd_step(swe_adj* A, const double* h, const double* qx, const double* qy, double* ho,
              double* qxo, double* qyo, double dt_fixed, int k, double* phi_out = nullptr,
              double* phi2_out = nullptr) {
    MemberArgs m = A->m;
    m.h[0] = (double*)h; m.qx[0] = (double*)qx; m.qy[0] = (double*)qy;
    m.h[1] = ho; m.qx[1] = qxo; m.qy[1] = qyo;
    m.dtlog = dt_fixed > 0.0 ? nullptr : A->dts + k;
    m.dtlog_cap = dt_fixed > 0.0 ? 0 : 1;
    if (phi_out) {
        m.ph = plane(phi_out, A->n, 0);
        m.pqx = plane(phi_out, A->n, 1);
        m.pqy = plane(phi_out, A->n, 2);
    }
    // the logged entry is indexed by the step count of the scalar block,
    // which is reset to 0 before each step so that dts[k] receives it; a
    // frozen dt reads neither the count nor the wave-speed bounds
    if (!(dt_fixed > 0.0))
        hipLaunchKernelGGL(reset_step_kernel, dim3(1), dim3(64), 0, A->stream, m.sc);
    TileIO io = host_step_io(m, 0, 0, INFINITY);
    io.dt_fixed = dt_fixed;
    launch_fwd<1>(A->prm, A->stream, m, io);
    if (phi2_out) {
        io.ph2 = plane(phi2_out, A->n, 0);
        io.pqx2 = plane(phi2_out, A->n, 1);
        io.pqy2 = plane(phi2_out, A->n, 2);
        launch_fwd<2, true>(A->prm, A->stream, m, io);
    } else {
        launch_fwd<2>(A->prm, A->stream, m, io);
    }
}

// Phi(U) into dst (stage 1 kernel with a scratch accumulator).
void rate_into(swe_adj* A, const double* h, const double* qx, const double* qy, double* dst) {
    MemberArgs m = A->m;
    TileIO io;
    std::memset(&io, 0, sizeof io);
    io.h = h; io.qx = qx; io.qy = qy;
    io.ph = plane(dst, A->n, 0);
    io.pqx = plane(dst, A->n, 1);
    io.pqy = plane(dst, A->n, 2);
    // the wave-speed bounds go to slot 2, which nothing reads here: it is
    // not cleared
    io.acc = &m.sc->amax[2][0][0];
    io.clr = nullptr;
    io.slot = 2;
    launch_fwd<1>(A->prm, A->stream, m, io);
}

// lam(h,qx,qy) += VJP_Phi(U, mu)
void vjp_rate(swe_adj* A, const double* h, const double* qx, const double* qy, double* lam) {
    const size_t n = A->n;
    const int nx = A->prm.nx, ny = A->prm.ny;
    const int ty = vjp_rows(nx, ny);
    dim3 grid((nx + VJP_TX - 7) / (VJP_TX - 6), (ny + ty - 1) / ty);
    double* mu = A->mu;
    if (A->prm.flux == 2)
        hipLaunchKernelGGL((adj_vjp_kernel<VJP_TX, 2>), grid, dim3(VJP_TX), 0, A->stream, A->aa,
                           h, qx, qy, (const double*)plane(mu, n, 0),
                           (const double*)plane(mu, n, 1), (const double*)plane(mu, n, 2),
                           plane(lam, n, 0), plane(lam, n, 1), plane(lam, n, 2), ty);
    else if (A->prm.flux == 1)
        hipLaunchKernelGGL((adj_vjp_kernel<VJP_TX, 1>), grid, dim3(VJP_TX), 0, A->stream, A->aa,
                           h, qx, qy, (const double*)plane(mu, n, 0),
                           (const double*)plane(mu, n, 1), (const double*)plane(mu, n, 2),
                           plane(lam, n, 0), plane(lam, n, 1), plane(lam, n, 2), ty);
    else
        hipLaunchKernelGGL((adj_vjp_kernel<VJP_TX, 0>), grid, dim3(VJP_TX), 0, A->stream, A->aa,
                           h, qx, qy, (const double*)plane(mu, n, 0),
                           (const double*)plane(mu, n, 1), (const double*)plane(mu, n, 2),
                           plane(lam, n, 0), plane(lam, n, 1), plane(lam, n, 2), ty);
}

// lamA <- adjoint of U^k given lam = adjoint of U^{k+1}; grad += dL/dn.
// phik, phi2k: Phi(U^k) and Phi(U*) kept from the segment recompute, or
// null to recompute them.
void adj_step(swe_adj* A, const double* Uk, double dt, double* grad, const double* phik,
              const double* phi2k) {
    const size_t n = A->n;
    const double* h = Uk;
    const double* qx = Uk + n;
    const double* qy = Uk + 2 * n;
    double* us = A->ust;
    // Phi(U^k) (kept for stage 1) and U*
    if (!phik) {
        rate_into(A, h, qx, qy, A->phi0);
        phik = A->phi0;
    }
    // stage 2 on U*: Phi(U*), then its friction reversed with output
    // adjoint lam/2
    if (!phi2k) {
        hipLaunchKernelGGL(stage_out_kernel, dim3(blocks(n)), dim3(T1), 0, A->stream, A->m.p,
                           A->m.fric, h, qx, qy, plane(phik, n, 0), plane(phik, n, 1),
                           plane(phik, n, 2), dt, plane(us, n, 0), plane(us, n, 1),
                           plane(us, n, 2), n);
        rate_into(A, plane(us, n, 0), plane(us, n, 1), plane(us, n, 2), A->phi);
        hipLaunchKernelGGL(adj_stage_kernel, dim3(blocks(n)), dim3(T1), 0, A->stream, A->m.p,
                           A->m.fric, (const double*)plane(us, n, 0),
                           (const double*)plane(us, n, 1), (const double*)plane(us, n, 2),
                           plane(A->phi, n, 0), plane(A->phi, n, 1), plane(A->phi, n, 2), dt,
                           (const double*)plane(A->lam, n, 0),
                           (const double*)plane(A->lam, n, 1),
                           (const double*)plane(A->lam, n, 2), 0.5, plane(A->lamB, n, 0),
                           plane(A->lamB, n, 1), plane(A->lamB, n, 2), 0, nullptr, nullptr,
                           nullptr, plane(A->mu, n, 0), plane(A->mu, n, 1), plane(A->mu, n, 2),
                           grad, n);
    } else {
        // U* rebuilt and stage 2 reversed in one pass
        hipLaunchKernelGGL(adj_stage2_kernel, dim3(blocks(n)), dim3(T1), 0, A->stream, A->m.p,
                           A->m.fric, h, qx, qy, plane(phik, n, 0), plane(phik, n, 1),
                           plane(phik, n, 2), plane(phi2k, n, 0), plane(phi2k, n, 1),
                           plane(phi2k, n, 2), dt, (const double*)plane(A->lam, n, 0),
                           (const double*)plane(A->lam, n, 1),
                           (const double*)plane(A->lam, n, 2), plane(us, n, 0), plane(us, n, 1),
                           plane(us, n, 2), plane(A->lamB, n, 0), plane(A->lamB, n, 1),
                           plane(A->lamB, n, 2), plane(A->mu, n, 0), plane(A->mu, n, 1),
                           plane(A->mu, n, 2), grad, n);
    }
    vjp_rate(A, plane(us, n, 0), plane(us, n, 1), plane(us, n, 2), A->lamB);
    // stage 1 on U^k: friction reversed with output adjoint lamB; lamA =
    // lam/2 (Heun: lam_n takes half of lam directly) + that
    hipLaunchKernelGGL(adj_stage_kernel, dim3(blocks(n)), dim3(T1), 0, A->stream, A->m.p,
                       A->m.fric, h, qx, qy, plane(phik, n, 0), plane(phik, n, 1),
                       plane(phik, n, 2), dt,
                       (const double*)plane(A->lamB, n, 0), (const double*)plane(A->lamB, n, 1),
                       (const double*)plane(A->lamB, n, 2), 1.0, plane(A->lamA, n, 0),
                       plane(A->lamA, n, 1), plane(A->lamA, n, 2), 2,
                       (const double*)plane(A->lam, n, 0), (const double*)plane(A->lam, n, 1),
                       (const double*)plane(A->lam, n, 2), plane(A->mu, n, 0),
                       plane(A->mu, n, 1), plane(A->mu, n, 2), grad, n);
    vjp_rate(A, h, qx, qy, A->lamA);
}

}  // namespace

extern "C" {

int swe_adj_workspace_bytes(const swe_params* p, int32_t nsteps, int32_t ckpt_every,
                            int32_t ngauges, int32_t every, size_t* bytes) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!bytes || nsteps < 1 || ckpt_every < 1 || ngauges < 0 || every < 1) return SWE_EINVAL;
    *bytes = adj_bytes(p, nsteps, ckpt_every, ngauges, every);
    return SWE_OK;
}

int swe_adj_create(const swe_params* p, const swe_buffers* b, int32_t nsteps,
                   int32_t ckpt_every, const int32_t* gauges, int32_t ngauges, int32_t every,
                   const double* obs, void* workspace, size_t workspace_bytes, void* stream,
                   swe_adj** out) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!b || !out || !workspace || !b->h || !b->qx || !b->qy || !b->z || !b->fric)
        return SWE_EINVAL;
    // the second-order scheme (any of the three fluxes)
    if (p->infil_on || p->fric_law == SWE_FRIC_NONE || p->order == 1) return SWE_EINVAL;
    // the reverse sweeps exist for MUSCL and the HLL, Rusanov and kinetic fluxes
    if (p->flux == 3 || p->recon != 0) return SWE_EINVAL;
    // walls and free outflow only: the reverse pass has no imposed ghosts
    for (int s = 0; s < 4; ++s)
        if (p->bc[s] >= SWE_BC_IMPOSED_H) return SWE_EINVAL;
    // uniform rain only: the reverse pass has no rain or soil fields
    if (b->rain_w || b->ks || b->psi || b->dtheta) return SWE_EINVAL;
    if (nsteps < 1 || ckpt_every < 1 || ngauges < 1 || every < 1 || !gauges || !obs)
        return SWE_EINVAL;
    if (((uintptr_t)workspace & 255) != 0) return SWE_EINVAL;
    const AdjLayout L = adj_layout(p, nsteps, ckpt_every, ngauges, every);
    if (workspace_bytes < L.total) return SWE_ENOMEM;
    {
        // every gauge must be a cell of the grid
        std::vector<int32_t> g(ngauges);
        if (hipMemcpy(g.data(), gauges, ngauges * sizeof(int32_t), hipMemcpyDeviceToHost) !=
            hipSuccess)
            return SWE_EHIP;
        for (int32_t v : g)
            if (v < 0 || (size_t)v >= ncells(p)) return SWE_EINVAL;
    }
    swe_adj* A = new (std::nothrow) swe_adj;
    if (!A) return SWE_ENOMEM;
    std::memset(A, 0, sizeof *A);
    A->prm = *p;
    A->stream = (hipStream_t)stream;
    A->nsteps = nsteps;
    A->every = every;
    A->ngauges = ngauges;
    A->ckpt = L.ckpt;
    A->nrows = nsteps / every;
    A->gauges = gauges;
    A->obs = obs;
    A->h0 = b->h; A->qx0 = b->qx; A->qy0 = b->qy;
    size_t n = ncells(p), an = align256(n * sizeof(double));
    A->n = n;
    char* const base = (char*)workspace;
    MemberArgs& m = A->m;
    m.p = to_kparams(*p);
    m.z = b->z;
    m.fric = b->fric;
    m.vinf = nullptr;
    m.sc = (DevScalars*)(base + L.scalars);
    A->loss_dev = (double*)(base + L.loss);
    A->dts = (double*)(base + L.dts);
    A->series = (double*)(base + L.series);
    A->ckpts = (double*)(base + L.ckpts);
    A->seg = (double*)(base + L.seg);
    A->segphi = (double*)(base + L.segphi);
    A->segphi2 = (double*)(base + L.segphi2);
    char* w = base + L.tail;
    A->ust = (double*)w; w += 3 * an;
    A->phi = (double*)w; w += 3 * an;
    A->phi0 = (double*)w; w += 3 * an;
    A->lamA = (double*)w; w += 3 * an;
    A->lamB = (double*)w; w += 3 * an;
    A->lam = (double*)w; w += 3 * an;
    A->mu = (double*)w; w += 3 * an;
    if ((size_t)(w - base) != L.total) {  // the carve-up is the layout
        delete A;
        return SWE_EINVAL;
    }
    A->aa.p = m.p;
    A->aa.z = b->z;
    A->aa.fric = b->fric;
    // the forward writes Phi into the same planes the rate kernel uses
    m.ph = plane(A->phi, n, 0);
    m.pqx = plane(A->phi, n, 1);
    m.pqy = plane(A->phi, n, 2);
    // the planes are laid out with stride n (not the aligned stride): keep
    // that consistent by allocating 3 * an >= 3 * n * 8 per triple
    hipLaunchKernelGGL(swe_init_scalars_kernel, dim3(1), dim3(64), 0, A->stream, m.sc, 0.0);
    rc = hip_ok(hipGetLastError());
    if (rc) { delete A; return rc; }
    *out = A;
    return SWE_OK;
}

int swe_adj_destroy(swe_adj* A) {
    delete A;
    return SWE_OK;
}

int swe_adj_set_dts(swe_adj* A, const double* dts) {
    if (!A) return SWE_EINVAL;
    A->last_kept = false;  // the kept segment belongs to the old steps
    if (!dts) {
        A->dts_frozen = false;
        return SWE_OK;
    }
    if (hipMemcpyAsync(A->dts, dts, A->nsteps * sizeof(double), hipMemcpyDeviceToDevice,
                       A->stream) != hipSuccess)
        return SWE_EHIP;
    A->dts_frozen = true;
    return SWE_OK;
}

int swe_adj_get_dts(swe_adj* A, double* dts) {
    if (!A || !dts) return SWE_EINVAL;
    if (hipMemcpyAsync(dts, A->dts, A->nsteps * sizeof(double), hipMemcpyDeviceToDevice,
                       A->stream) != hipSuccess)
        return SWE_EHIP;
    return SWE_OK;
}

int swe_adj_get_series(swe_adj* A, double* out) {
    if (!A || !out) return SWE_EINVAL;
    if (hipMemcpyAsync(out, A->series, (size_t)A->nrows * A->ngauges * sizeof(double),
                       hipMemcpyDeviceToDevice, A->stream) != hipSuccess)
        return SWE_EHIP;
    return SWE_OK;
}

int swe_adj_forward(swe_adj* A, double* loss) {
    Range range("swe_adj_forward");
    if (!A) return SWE_EINVAL;
    const size_t n = A->n;
    // state ping-pong in the segment buffer's first two slots
    double* S0 = A->seg;
    double* S1 = A->seg + 3 * n;
    (void)hipMemcpyAsync(S0, A->h0, n * sizeof(double), hipMemcpyDeviceToDevice, A->stream);
    (void)hipMemcpyAsync(S0 + n, A->qx0, n * sizeof(double), hipMemcpyDeviceToDevice, A->stream);
    (void)hipMemcpyAsync(S0 + 2 * n, A->qy0, n * sizeof(double), hipMemcpyDeviceToDevice, A->stream);
    std::vector<double> host_dts;
    if (A->dts_frozen) {
        host_dts.resize(A->nsteps);
        if (hipMemcpyAsync(host_dts.data(), A->dts, A->nsteps * sizeof(double),
                           hipMemcpyDeviceToHost, A->stream) != hipSuccess)
            return SWE_EHIP;
        if (hipStreamSynchronize(A->stream) != hipSuccess) return SWE_EHIP;
    }
    double* cur = S0;
    double* nxt = S1;
    // the last segment's steps write their states and both rates where the
    // backward pass's recompute of that segment would, which it then skips
    // (with one segment, ckpt_every >= nsteps, the reverse recomputes nothing)
    const int last = ((A->nsteps - 1) / A->ckpt) * A->ckpt;
    A->last_kept = false;
    for (int k = 0; k < A->nsteps; ++k) {
        if (k % A->ckpt == 0)
            (void)hipMemcpyAsync(A->ckpts + (size_t)(k / A->ckpt) * 3 * n, cur, 3 * n * sizeof(double),
                           hipMemcpyDeviceToDevice, A->stream);
        double *phi = nullptr, *phi2 = nullptr;
        if (k >= last) {
            if (k == last && cur != S0) {
                (void)hipMemcpyAsync(S0, cur, 3 * n * sizeof(double), hipMemcpyDeviceToDevice,
                                     A->stream);
                cur = S0;
            }
            nxt = cur + 3 * n;
            phi = A->segphi + (size_t)(k - last) * 3 * n;
            phi2 = A->segphi2 + (size_t)(k - last) * 3 * n;
        }
        fwd_step(A, cur, cur + n, cur + 2 * n, nxt, nxt + n, nxt + 2 * n,
                 A->dts_frozen ? host_dts[k] : 0.0, k, phi, phi2);
        if ((k + 1) % A->every == 0 && (k + 1) / A->every <= A->nrows)
            hipLaunchKernelGGL(gauge_kernel, dim3((A->ngauges + 63) / 64), dim3(64), 0,
                               A->stream, (const double*)nxt, A->gauges, A->ngauges,
                               A->series + (size_t)((k + 1) / A->every - 1) * A->ngauges);
        if (k >= last) {
            cur = nxt;
        } else {
            double* t = cur; cur = nxt; nxt = t;
        }
    }
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(64), 0, A->stream, (const double*)A->series,
                       A->obs, (size_t)A->nrows * A->ngauges, A->loss_dev);
    double l = 0.0;
    if (hipMemcpyAsync(&l, A->loss_dev, sizeof l, hipMemcpyDeviceToHost, A->stream) != hipSuccess)
        return SWE_EHIP;
    if (hipStreamSynchronize(A->stream) != hipSuccess) return SWE_EHIP;
    DevScalars s;
    if (hipMemcpy(&s, A->m.sc, sizeof s, hipMemcpyDeviceToHost) != hipSuccess) return SWE_EHIP;
    if (loss) *loss = l;
    A->dts_frozen = true;  // the backward pass replays exactly these steps
    A->last_kept = true;
    if (s.status & SWE_FLAG_NONFINITE) return SWE_ENONFINITE;
    if (s.status & SWE_FLAG_NEGDEPTH) return SWE_ENEGDEPTH;
    if (s.status & SWE_FLAG_DT) return SWE_EDT;
    if (s.status & SWE_FLAG_DT_UNDERFLOW) return SWE_EDTMIN;
    return hip_ok(hipGetLastError());
}

int swe_adj_backward(swe_adj* A, double* grad) {
    Range range("swe_adj_backward");
    if (!A || !grad) return SWE_EINVAL;
    const size_t n = A->n;
    std::vector<double> dts(A->nsteps);
    if (hipMemcpyAsync(dts.data(), A->dts, A->nsteps * sizeof(double), hipMemcpyDeviceToHost,
                       A->stream) != hipSuccess)
        return SWE_EHIP;
    if (hipStreamSynchronize(A->stream) != hipSuccess) return SWE_EHIP;
    hipLaunchKernelGGL(fill_kernel, dim3(1024), dim3(256), 0, A->stream, grad, 0.0, n);
    hipLaunchKernelGGL(fill_kernel, dim3(1024), dim3(256), 0, A->stream, A->lam, 0.0, 3 * n);
    const int nseg = (A->nsteps + A->ckpt - 1) / A->ckpt;
    for (int sg = nseg - 1; sg >= 0; --sg) {
        const int s = sg * A->ckpt;
        const int e = s + A->ckpt < A->nsteps ? s + A->ckpt : A->nsteps;
        // the forward pass left the last segment in place, rates included
        const bool full = sg == nseg - 1 && A->last_kept;
        // else recompute U^s .. U^{e-1} into the segment buffer
        if (!full) {
            (void)hipMemcpyAsync(A->seg, A->ckpts + (size_t)sg * 3 * n, 3 * n * sizeof(double),
                                 hipMemcpyDeviceToDevice, A->stream);
            A->last_kept = false;
        }
        for (int k = s; !full && k < e - 1; ++k) {
            double* in = A->seg + (size_t)(k - s) * 3 * n;
            double* o = in + 3 * n;
            fwd_step(A, in, in + n, in + 2 * n, o, o + n, o + 2 * n, dts[k], k,
                     A->segphi + (size_t)(k - s) * 3 * n, A->segphi2 + (size_t)(k - s) * 3 * n);
        }
        for (int k = e - 1; k >= s; --k) {
            // loss term of U^{k+1}
            if ((k + 1) % A->every == 0 && (k + 1) / A->every <= A->nrows) {
                size_t row = (size_t)((k + 1) / A->every - 1) * A->ngauges;
                hipLaunchKernelGGL(inject_kernel, dim3(1), dim3(64), 0, A->stream,
                                   (const double*)(A->series + row), A->obs + row, A->gauges,
                                   A->ngauges, A->lam);
            }
            const double* Uk = A->seg + (size_t)(k - s) * 3 * n;
            // the recompute stops before the segment's last step; the
            // forward pass did not
            const bool kept = full || k < e - 1;
            adj_step(A, Uk, dts[k], grad, kept ? A->segphi + (size_t)(k - s) * 3 * n : nullptr,
                     kept ? A->segphi2 + (size_t)(k - s) * 3 * n : nullptr);
            // lam <- lamA (the buffers trade places)
            std::swap(A->lam, A->lamA);
        }
    }
    if (hipStreamSynchronize(A->stream) != hipSuccess) return SWE_EHIP;
    return hip_ok(hipGetLastError());
}

}  // extern "C"
