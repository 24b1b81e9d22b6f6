// Device code shared by the single-simulation and the ensemble kernels:
// the formulas of the scheme (arXiv:1307.4839, Sections 2-3) and the
// routine that advances one tile (a strip of columns over a range of rows)
// through one stage.
//
// Tiling: a block of TXT threads owns a strip of TXT columns, of which the
// TXT-4 interior ones are outputs (two halo columns per side feed the
// second-order stencil), and marches down a range of rows.  Along y the
// stencil lives in registers (each thread keeps a rolling window of its own
// column, and the loads of the next row are issued one iteration ahead), so
// every y-face is evaluated once.  Along x neighbours exchange values
// through LDS, so every x-face is also evaluated once.  Boundary ghost cells
// (Section 2.2, two layers at second order, Section 6.1) are index maps in
// the loader; no ghost arrays exist in HBM.
//
// Arithmetic follows the formulas in the order they are written, without
// contraction; divisions and square roots give the values of the IEEE
// operators (see Division), so the only operation that is not correctly
// rounded is the cube root of the Manning law.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "swe.h"

namespace swe_dev {

constexpr int HALO = 2;  // ghost/halo width at second order

// ---------------------------------------------------------------------------
// Device-side scalars (in the workspace)
// ---------------------------------------------------------------------------

// The wave-speed maxima of a step are accumulated in AMAX_SPREAD pairs
// (Ax, Ay), each on its own 128-byte line: the stage-1 block with spread
// index b folds its maxima into pair b mod AMAX_SPREAD, so that thousands of
// blocks finishing together do not queue on one address; readers take the
// maximum over the pairs (the same value: max is associative).
constexpr int AMAX_SPREAD = 16;
constexpr int AMAX_LINE = 16;  // unsigned long long per 128-byte line

static_assert(SWE_HYETO_MAX <= 128, "the hyetograph lookup counts with two wave64 ballots");

struct DevScalars {
    // per slot: bit patterns of Ax, Ay >= 0 at [pair][0], [pair][1]
    unsigned long long amax[3][AMAX_SPREAD][AMAX_LINE];
    double t[2];                    // time, double-buffered by step parity
    long long steps[2];             // steps taken, double-buffered
    double last_dt;
    unsigned int status;            // sticky SWE_FLAG_* bits
    unsigned int pad;
    double rain_depth;              // sum over the steps taken of dt r(t^n)
    double water0;                  // sum of h + V_inf when the context was made
    // hyetograph r(t): hy_r[k] from hy_t[k] (strictly increasing) up to the
    // next breakpoint, 0 before hy_t[0]; hy_n = 0: the constant rain of the
    // parameters
    int hy_n;
    int hy_pad;
    double hy_t[SWE_HYETO_MAX];
    double hy_r[SWE_HYETO_MAX];
};
// bytes a scalar block takes in a workspace (a multiple of 256)
constexpr size_t SCALAR_BYTES = (sizeof(DevScalars) + 255) / 256 * 256;

struct KParams {
    int nx, ny;
    double dx, dy, g, cfl, dt_max, h_eps;
    // a dt of eq. (cfl) below dt_min (other than the step clipped to the end
    // time) is a collapse: the step is not taken
    double dt_min;
    int bcw, bce, bcs, bcn;
    int law;
    double coef;
    double rain;
    int infil;
    double ks, psi, dtheta;
    // dx and dy both powers of two: X / dx == X * inv_dx exactly
    int dxy_pow2;
    double inv_dx, inv_dy;
    // g in (0, 2^10] and dx, dy in [2^-300, 2^300]: the shared-reciprocal
    // quotients may be used (their operand bounds are checked on the device)
    int fast_div;
    // 2: MUSCL + Heun; 1: first order (no reconstruction, one Euler stage)
    int order;
    // second-order reconstruction: 0 MUSCL, 1 ENO, 2 modified ENO
    int recon;
    // 0: HLL; 1: Rusanov; 2: kinetic; 3: VFRoe-ncv
    int flux;
    // some side has an imposed depth or discharge; its values per side
    // (west, east, south, north)
    int imposed;
    double bc_h[4], bc_q[4];
};

// ---------------------------------------------------------------------------
// Division
// ---------------------------------------------------------------------------
//
// On gfx9 a / b in double precision is: operand scaling, a reciprocal seed
// of b, two Newton-Raphson steps y <- y + y (1 - b y), the quotient
// q0 = a y, the exact residual r = a - b q0, the corrected quotient
// q0 + r y, and a special-case fix-up.  The scaling and the fix-up only act
// on zero, non-finite, tiny or huge operands: for b in [2^-300, 2^300] and
// a in [2^-700, 2^460] neither does, the corrected quotient is the result of
// the division operator, and the refined reciprocal depends on b alone.  It
// can then be computed once per denominator and shared by every numerator
// over it: three operations per quotient instead of eleven.  A zero
// numerator gives a zero quotient (its sign may differ from the operator's;
// nothing in the scheme tells the two zeros apart).
//
// The formulas take a division policy.  ExactDiv is the division operator.
// FastDiv shares reciprocals and, without branches, keeps two running
// bounds over the operands it is shown: the largest magnitude among the
// capped values, and the smallest binary exponent among the values bounded
// below (a zero counts as exponent 0, a depth with its sign bit set as a
// huge negative exponent).  While every capped value stays at most 2^60 and
// every value bounded below is zero or at least 2^-300, every operand of a
// shared-reciprocal quotient lies in the window above, and so does every
// operand of a square root without scaling (root); the comments at each
// quotient give the reason.  The tile kernel checks the bounds once per row
// and, when they fail, computes the row again with ExactDiv, as it does
// every later row of the tile.

struct Recip {
    double b, y;  // denominator and its refined reciprocal (FastDiv only)
};

constexpr double NOTE_CAP = 0x1p60;
constexpr int NOTE_EMIN = -299;  // frexp exponent of 2^-300

struct ExactDiv {
    __host__ __device__ Recip rcp(double b) const { return Recip{b, 0.0}; }
    __host__ __device__ double div(double a, const Recip& r) const { return a / r.b; }
    __host__ __device__ void cap(double) const {}
    __host__ __device__ void low(double) const {}
    __host__ __device__ void low2(double, double) const {}
    __host__ __device__ void depth(double) const {}
    __host__ __device__ double root(double x) const { return sqrt(x); }
    __host__ __device__ bool ok() const { return true; }
    __host__ __device__ void settle() const {}
};

struct FastDiv {
    double hi = 0.0;  // largest magnitude among the capped values
    int emin = 0;     // smallest exponent among the values bounded below

    __device__ Recip rcp(double b) const {
        double y = __builtin_amdgcn_rcp(b);
        double e = fma(-b, y, 1.0);
        y = fma(y, e, y);
        e = fma(-b, y, 1.0);
        return Recip{b, fma(y, e, y)};
    }
    __device__ double div(double a, const Recip& r) const {
        double q0 = a * r.y;
        double e = fma(-r.b, q0, a);
        return fma(e, r.y, q0);
    }
    // Square root as gfx9 evaluates it for x = 0, x >= 2^-767, +inf, x < 0
    // and NaN (reciprocal square root seed, Goldschmidt steps for g ~ sqrt(x)
    // and h ~ 1 / (2 sqrt(x)), two corrections with the exact residual
    // x - g^2, zero and infinity returned as they are), without the scaling
    // by 2^256 that only positive x below 2^-767 take: the caller bounds x
    // below.
    __device__ double root(double x) const {
        double r = __builtin_amdgcn_rsq(x);
        double g = x * r;
        double h = r * 0.5;
        double e = fma(-h, g, 0.5);
        g = fma(g, e, g);
        h = fma(h, e, h);
        double d = fma(-g, g, x);
        g = fma(d, h, g);
        d = fma(-g, g, x);
        g = fma(d, h, g);
        return (x == 0.0 || x == __builtin_inf()) ? x : g;
    }
    __device__ void cap(double v) { hi = fmax(hi, fabs(v)); }
    __device__ void low(double v) { emin = min(emin, __builtin_amdgcn_frexp_exp(v)); }
    __device__ void low2(double u, double v) {
        emin = min(emin, min(__builtin_amdgcn_frexp_exp(u), __builtin_amdgcn_frexp_exp(v)));
    }
    // a depth: capped, bounded below, and not negative (the high word of a
    // double with its sign bit set is a negative integer)
    __device__ void depth(double h) {
        cap(h);
        emin = min(emin, min(__builtin_amdgcn_frexp_exp(h), __double2hiint(h)));
    }
    __device__ bool ok() const { return hi <= NOTE_CAP && emin >= NOTE_EMIN; }
    // Pins the bounds at this point of the program, so that the values
    // shown before it need not stay live until the row's check.
    __device__ void settle() { asm volatile("" : "+v"(hi), "+v"(emin)); }
};

// ---------------------------------------------------------------------------
// Formulas (Sections 3.1, 3.3, 3.4)
// ---------------------------------------------------------------------------

// For ordered (non-NaN) operands these return the same value as the
// comparisons they replace (up to the sign of a zero, which no later
// operation can turn into a different non-zero value).
__host__ __device__ __forceinline__ double vmax(double a, double b) { return fmax(a, b); }
__host__ __device__ __forceinline__ double vmin(double a, double b) { return fmin(a, b); }

// minmod limiter, Section 3.4: min(a, b) if both >= 0, max(a, b) if both
// <= 0, else 0.  Branch-free form with the same value:
// max(min(a, b), min(max(a, b), 0)).
__host__ __device__ __forceinline__ double minmod(double a, double b) {
    return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
}

// primitive variables of a cell: depth, velocity normal and tangential to
// the sweep direction, free surface eta = h + z
struct Prim {
    double h, un, ut, eta;
};

// reconstructed face values: _m at the face i-1/2, _p at the face i+1/2
struct Rec {
    double h_m, h_p, z_m, z_p, un_m, un_p, ut_m, ut_p;
};

// MUSCL on h, h+z and the velocity with minmod on undivided differences;
// z deduced; modified velocity reconstruction conserving discharge
// (Section 3.4).  A cell at or below the dry threshold keeps its velocity.
// rc = d.rcp(c.h).  With the three depths not negative, minmod keeps h_m and
// h_p within [c.h / 2, 3 c.h / 2] (up to one rounding), so the two quotients
// need no operand bounds beyond those of c.h.
template <class D>
__host__ __device__ __forceinline__ Rec muscl(const Prim& a, const Prim& c, const Prim& b,
                                              double h_eps, const Recip& rc, D& d) {
    Rec r;
    double dh = minmod(c.h - a.h, b.h - c.h);
    r.h_m = c.h - 0.5 * dh;
    r.h_p = c.h + 0.5 * dh;
    double de = minmod(c.eta - a.eta, b.eta - c.eta);
    double eta_m = c.eta - 0.5 * de;
    double eta_p = c.eta + 0.5 * de;
    r.z_m = eta_m - r.h_m;
    r.z_p = eta_p - r.h_p;
    double dun = minmod(c.un - a.un, b.un - c.un);
    double dut = minmod(c.ut - a.ut, b.ut - c.ut);
    if (c.h > h_eps) {
        double wp = d.div(r.h_p, rc);
        double wm = d.div(r.h_m, rc);
        r.un_m = c.un - wp * (0.5 * dun);
        r.un_p = c.un + wm * (0.5 * dun);
        r.ut_m = c.ut - wp * (0.5 * dut);
        r.ut_p = c.ut + wm * (0.5 * dut);
    } else {
        r.un_m = c.un;
        r.un_p = c.un;
        r.ut_m = c.ut;
        r.ut_p = c.ut;
    }
    return r;
}

__host__ __device__ __forceinline__ Rec muscl(const Prim& a, const Prim& c, const Prim& b,
                                              double h_eps) {
    ExactDiv d;
    return muscl(a, c, b, h_eps, d.rcp(c.h), d);
}

// ENO at second order (Section 4.1 names ENO and modified ENO beside MUSCL;
// the paper's second-order stencils are the cells i-1, i, i+1): the slope of
// h, h+z and the velocities is the one-sided undivided difference of smaller
// magnitude (the left one on ties).  A cell at or below the dry threshold
// keeps its values at both faces.  MOD (modified ENO): the depth's slope is
// limited to |D| <= 2 h, so both face depths stay in [0, 2 h].  Unlike
// minmod's, the face depths may be anywhere (negative with plain ENO), so
// the two quotients bound their numerators.
__host__ __device__ __forceinline__ double eno_slope(double a, double b) {
    return fabs(a) <= fabs(b) ? a : b;
}

template <bool MOD, class D>
__host__ __device__ __forceinline__ Rec eno(const Prim& a, const Prim& c, const Prim& b,
                                            double h_eps, const Recip& rc, D& d) {
    Rec r;
    if (!(c.h > h_eps)) {
        r.h_m = r.h_p = c.h;
        r.z_m = r.z_p = c.eta - c.h;
        r.un_m = r.un_p = c.un;
        r.ut_m = r.ut_p = c.ut;
        return r;
    }
    double dh = eno_slope(c.h - a.h, b.h - c.h);
    if (MOD) {
        const double cap = 2.0 * c.h;
        dh = fmin(fmax(dh, -cap), cap);
    }
    r.h_m = c.h - 0.5 * dh;
    r.h_p = c.h + 0.5 * dh;
    double de = eno_slope(c.eta - a.eta, b.eta - c.eta);
    double eta_m = c.eta - 0.5 * de;
    double eta_p = c.eta + 0.5 * de;
    r.z_m = eta_m - r.h_m;
    r.z_p = eta_p - r.h_p;
    double dun = eno_slope(c.un - a.un, b.un - c.un);
    double dut = eno_slope(c.ut - a.ut, b.ut - c.ut);
    d.cap(r.h_m);
    d.cap(r.h_p);
    d.low2(r.h_m, r.h_p);
    d.settle();
    double wp = d.div(r.h_p, rc);
    double wm = d.div(r.h_m, rc);
    r.un_m = c.un - wp * (0.5 * dun);
    r.un_p = c.un + wm * (0.5 * dun);
    r.ut_m = c.ut - wp * (0.5 * dut);
    r.ut_p = c.ut + wm * (0.5 * dut);
    return r;
}

// Face values of a cell: ORDER 2 MUSCL, 3 ENO, 4 modified ENO (all second
// order); at first order (ORDER 1, Section 3.3) the cell's own values, i.e.
// the reconstruction above with zero slopes (z still deduced from h and
// h+z).
template <int ORDER, class D>
__host__ __device__ __forceinline__ Rec reconstruct(const Prim& a, const Prim& c, const Prim& b,
                                                    double h_eps, const Recip& rc, D& d) {
    if constexpr (ORDER == 1) {
        Rec r;
        r.h_m = r.h_p = c.h;
        r.z_m = r.z_p = c.eta - c.h;
        r.un_m = r.un_p = c.un;
        r.ut_m = r.ut_p = c.ut;
        return r;
    } else if constexpr (ORDER == 3 || ORDER == 4) {
        return eno<ORDER == 4>(a, c, b, h_eps, rc, d);
    } else {
        return muscl(a, c, b, h_eps, rc, d);
    }
}

// Flux through one face: hydrostatic reconstruction (Section 3.1), HLL
// (Section 3.3; FLUX 1: the Rusanov flux, FLUX 2: the kinetic flux, two
// other consistent fluxes that section lists), and the normal-momentum
// corrections S_L (left cell) and S_R (right cell).  fl = flux seen by the
// left cell, fr = by the right one.  face_speed = max(|u-| + sqrt(g h-),
// |u+| + sqrt(g h+)) on the MUSCL states (stage 1 only); with the kinetic
// flux, g is replaced by 3g/2 (the particles' largest speed).
struct FaceOut {
    double f0, fl1, fr1, f2;
};

// Kinetic flux (Perthame and Simeoni, 2001): one side's share.  The state
// (h, u) is the mean of particles with velocities uniform on [u - s, u + s],
// s = sqrt(3 g h / 2), density h / (2 s); the left state sends those with
// xi > 0, the right one those with xi < 0.  m0 = int xi M = h (b^2 - a^2) /
// (4 s) and m1 = int xi^2 M = h (b^3 - a^3) / (6 s) over the part [a, b] of
// the support on the sending side; a dry side sends nothing.  Plain
// quotients and roots (correctly rounded), no shared reciprocals.
template <bool LEFT>
__host__ __device__ __forceinline__ void kinetic_half(double g, double h, double un, double& m0,
                                                      double& m1) {
    const double s = sqrt((1.5 * g) * h);
    double a = un - s;
    double b = un + s;
    if (LEFT) {
        a = fmax(a, 0.0);
        b = fmax(b, 0.0);
    } else {
        a = fmin(a, 0.0);
        b = fmin(b, 0.0);
    }
    const double n0 = h * (b * b - a * a);
    const double n1 = h * (b * b * b - a * a * a);
    const bool wet = h > 0.0;
    m0 = wet ? n0 / (4.0 * s) : 0.0;
    m1 = wet ? n1 / (6.0 * s) : 0.0;
}

// With depths, velocities and z capped at 2^60 and g at most 2^10, c1 and c2
// stay below 2^62 and the HLL numerators below 2^251; den and the
// numerators are bounded below here.  The Rusanov flux divides by nothing.
// FLUX 3: the VFRoe-ncv flux, the interface value of the Riemann problem in
// (2c, u) linearized about the mean state (U_L if uh - ch >= 0, U_R if
// uh + ch <= 0, else c* = ch + (uL - uR)/4, u* = uh + (cL - cR) and
// h* = max(c*, 0)^2 / g), the tangential velocity upwinded on u*; a dry side
// takes the other side's velocity and two dry sides pass nothing.  Its one
// quotient, c*^2 / g, is the division operator (g is not bounded below by
// the fast window).
template <int FLUX = 0, class D>
__host__ __device__ __forceinline__ FaceOut face(double g, double hm, double zm, double unm,
                                                 double utm, double hp, double zp, double unp,
                                                 double utp, D& d) {
    double zs = vmax(zm, zp);
    double hL = vmax(hm + zm - zs, 0.0);
    double hR = vmax(hp + zp - zs, 0.0);
    double gL = g * hL, gR = g * hR;
    d.low2(gL, gR);
    double cL = d.root(gL);
    double cR = d.root(gR);
    double c1 = vmin(unm - cL, unp - cR);
    double c2 = vmax(unm + cL, unp + cR);
    double qL = hL * unm;
    double qR = hR * unp;
    double hg = 0.5 * g;
    double FL0 = qL, FL1 = qL * unm + hg * hL * hL, FL2 = qL * utm;
    double FR0 = qR, FR1 = qR * unp + hg * hR * hR, FR2 = qR * utp;
    double F0, F1, F2;
    if constexpr (FLUX == 2) {
        double m0L, m1L, m0R, m1R;
        kinetic_half<true>(g, hL, unm, m0L, m1L);
        kinetic_half<false>(g, hR, unp, m0R, m1R);
        F0 = m0L + m0R;
        F1 = m1L + m1R;
        F2 = m0L * utm + m0R * utp;
    } else if constexpr (FLUX == 3) {
        const bool wL = hL > 0.0, wR = hR > 0.0;
        const double uL = wL ? unm : unp;
        const double uR = wR ? unp : unm;
        const double uh = 0.5 * (uL + uR);
        const double ch = 0.5 * (cL + cR);
        double hs, us;
        if (uh - ch >= 0.0) {
            hs = hL;
            us = uL;
        } else if (uh + ch <= 0.0) {
            hs = hR;
            us = uR;
        } else {
            const double cs = fmax(ch + 0.25 * (uL - uR), 0.0);
            hs = (cs * cs) / g;
            us = uh + (cL - cR);
        }
        const double qs = hs * us;
        const bool any = wL || wR;
        F0 = any ? qs : 0.0;
        F1 = any ? qs * us + hg * hs * hs : 0.0;
        F2 = any ? qs * (us >= 0.0 ? utm : utp) : 0.0;
    } else if constexpr (FLUX == 1) {
        // (F(U_L) + F(U_R))/2 - c/2 (U_R - U_L), c the largest local speed
        double c = vmax(fabs(unm) + cL, fabs(unp) + cR);
        F0 = 0.5 * (FL0 + FR0) - 0.5 * c * (hR - hL);
        F1 = 0.5 * (FL1 + FR1) - 0.5 * c * (qR - qL);
        F2 = 0.5 * (FL2 + FR2) - 0.5 * c * (hR * utp - hL * utm);
    } else if (0.0 <= c1) {
        F0 = FL0; F1 = FL1; F2 = FL2;
    } else if (c2 <= 0.0) {
        F0 = FR0; F1 = FR1; F2 = FR2;
    } else {
        Recip den = d.rcp(c2 - c1);
        double n0 = c1 * c2;
        double n1 = c2 * FL0 - c1 * FR0;
        double n2 = c2 * FL1 - c1 * FR1;
        double n3 = c2 * FL2 - c1 * FR2;
        d.low2(den.b, n0);
        d.low2(n1, n2);
        d.low(n3);
        d.settle();
        double w = d.div(n0, den);
        F0 = d.div(n1, den) + w * (hR - hL);
        F1 = d.div(n2, den) + w * (qR - qL);
        F2 = d.div(n3, den) + w * (hR * utp - hL * utm);
    }
    double sL = hg * (hm * hm - hL * hL);
    double sR = hg * (hp * hp - hR * hR);
    FaceOut o;
    o.f0 = F0;
    o.fl1 = F1 + sL;
    o.fr1 = F1 + sR;
    o.f2 = F2;
    return o;
}

template <int FLUX, class D>
__device__ __forceinline__ double face_speed(double g, double hm, double unm, double hp,
                                             double unp, D& d) {
    const double gs = FLUX == 2 ? 1.5 * g : g;
    double gm = gs * hm, gp = gs * hp;
    d.low2(gm, gp);
    double sm = fabs(unm) + d.root(gm);
    double sp = fabs(unp) + d.root(gp);
    return fmax(sm, sp);
}

__host__ __device__ __forceinline__ FaceOut face(double g, double hm, double zm, double unm,
                                                 double utm, double hp, double zp, double unp,
                                                 double utp) {
    ExactDiv d;
    return face(g, hm, zm, unm, utm, hp, zp, unp, utp, d);
}

// centred source Fc of Section 3.1 (normal momentum)
__host__ __device__ __forceinline__ double centred(double g, const Rec& r) {
    return (-g) * (0.5 * (r.h_m + r.h_p)) * (r.z_p - r.z_m);
}

// Semi-implicit friction of one stage (Section 3.2).  (h0, q0) stage input,
// (h1, q1) convective output.  The denominator and both numerators are
// capped and bounded below here, the operand of the square root too.
template <class D>
__host__ __device__ __forceinline__ void friction(const KParams& p, double coef, double h0,
                                                  double qx0, double qy0, double h1,
                                                  double& qx1, double& qy1, double dt, D& d) {
    if (h1 <= p.h_eps) {
        qx1 = 0.0;
        qy1 = 0.0;
        return;
    }
    if (p.law == SWE_FRIC_NONE || !(h0 > p.h_eps)) return;
    double q2 = qx0 * qx0 + qy0 * qy0;
    d.low(q2);
    double qn = d.root(q2);
    double den;
    if (p.law == SWE_FRIC_DARCY)
        den = 1.0 + dt * (coef / 8.0) * qn / (h0 * h1);
    else
        den = 1.0 + dt * p.g * coef * coef * qn / (h0 * (h1 * cbrt(h1)));
    Recip rd = d.rcp(den);
    d.cap(den);
    d.cap(qx1);
    d.cap(qy1);
    d.low2(den, qx1);
    d.low(qy1);
    d.settle();
    qx1 = d.div(qx1, rd);
    qy1 = d.div(qy1, rd);
}

__host__ __device__ __forceinline__ void friction(const KParams& p, double coef, double h0,
                                                  double qx0, double qy0, double h1,
                                                  double& qx1, double& qy1, double dt) {
    ExactDiv d;
    friction(p, coef, h0, qx0, qy0, h1, qx1, qy1, dt, d);
}

// dt from the wave-speed bounds (eq. cfl in 2D), clipped to dt_max and to
// the remaining time.
__host__ __device__ __forceinline__ double time_step(const KParams& p, double ax, double ay,
                                            double t, double t_end) {
    double r = ax / p.dx + ay / p.dy;
    double dt = p.dt_max;
    if (r > 0.0) {
        double c = p.cfl / r;
        if (c < dt) dt = c;
    }
    double rest = t_end - t;
    if (rest < dt) dt = rest;
    return dt;
}

// Rain at `rate` (the cell's R), then Green-Ampt (Section 3.5) with the
// cell's soil parameters; the infiltrated water leaves with the cell's
// velocity.
__host__ __device__ __forceinline__ void rain_infiltration(const KParams& p, double dt,
                                                  double rate, double ks, double psi,
                                                  double dtheta, double& h, double& qx,
                                                  double& qy, double& vinf) {
    h = h + dt * rate;
    if (!p.infil) return;
    double d;
    if (vinf > 0.0) {
        double zf = vinf / dtheta;
        double ic = ks * (1.0 + (psi + h) / zf);
        d = vmin(h, dt * ic);
    } else {
        d = h;
    }
    double h_old = h;
    h = h - d;
    vinf = vinf + d;
    if (h_old > 0.0) {
        double r = h / h_old;
        qx = qx * r;
        qy = qy * r;
    }
}

// ---------------------------------------------------------------------------
// Ghost mapping (Section 2.2): wall = mirror with negated normal discharge;
// outflow = copy of the boundary cell.
// ---------------------------------------------------------------------------

__host__ __device__ __forceinline__ int map_index(int c, int n, int bc_lo, int bc_hi,
                                         double& sign) {
    sign = 1.0;
    int s = c;
    if (c < 0) {
        if (bc_lo == SWE_BC_WALL) { s = -1 - c; sign = -1.0; }
        else s = 0;
    } else if (c >= n) {
        if (bc_hi == SWE_BC_WALL) { s = 2 * n - 1 - c; sign = -1.0; }
        else s = n - 1;
    }
    // indices beyond the two ghost layers are never used by an output;
    // keep them in bounds
    s = s < 0 ? 0 : (s >= n ? n - 1 : s);
    return s;
}

// ---------------------------------------------------------------------------
// Arguments
// ---------------------------------------------------------------------------

// One simulation (a member of an ensemble, or the single simulation of a
// context).  Read-only during a step.
struct MemberArgs {
    KParams p;
    const double* z;
    const double* fric;    // per-cell coefficient or nullptr
    double* vinf;          // Green-Ampt state or nullptr
    double* h[2];          // state buffers: [0] caller's, [1] workspace
    double* qx[2];
    double* qy[2];
    double* ph;            // stage rate Phi (3 arrays)
    double* pqx;
    double* pqy;
    DevScalars* sc;
    double* dtlog;
    long long dtlog_cap;
    // optional per-cell fields (nullptr: the scalar of the parameters):
    // rain weight w (R = r(t) w), Green-Ampt K_s, psi, theta_s - theta_i
    const double* rain_w;
    const double* ks_f;
    const double* psi_f;
    const double* dth_f;
};

// Buffers of one stage launch.
struct TileIO {
    const double* h;       // U^n
    const double* qx;
    const double* qy;
    double* ph;            // stage 1 writes, stage 2 reads
    double* pqx;
    double* pqy;
    double* ho;            // stage 2 output U^{n+1}
    double* qxo;
    double* qyo;
    unsigned long long* acc;  // stage 1: the (Ax, Ay) accumulators of the step (pairs)
    unsigned long long* clr;  // stage 1: accumulators zeroed for the next step (or null)
    int slot;                 // step parity (time buffer, accumulator slot)
    double t_end;
    double dt_fixed;          // > 0: use this time step instead of the CFL bound
    double* ph2;              // stage 2 with PHI2 only: Phi(U*) out
    double* pqx2;
    double* pqy2;
};

__device__ __forceinline__ TileIO step_io(const MemberArgs& m, int phase, int slot,
                                          double t_end) {
    TileIO io;
    io.h = m.h[phase];
    io.qx = m.qx[phase];
    io.qy = m.qy[phase];
    io.ph = m.ph;
    io.pqx = m.pqx;
    io.pqy = m.pqy;
    io.ho = m.h[phase ^ 1];
    io.qxo = m.qx[phase ^ 1];
    io.qyo = m.qy[phase ^ 1];
    io.acc = &m.sc->amax[slot][0][0];
    io.clr = &m.sc->amax[slot ^ 1][0][0];
    io.slot = slot;
    io.t_end = t_end;
    io.dt_fixed = 0.0;
    io.ph2 = io.pqx2 = io.pqy2 = nullptr;
    return io;
}

struct RawCell {
    double h, qx, qy, z;
};

// Raw values of one cell of the stage input as read from HBM.  Stage 1:
// U^n and z.  Stage 2 also: Phi(U^n) and the friction coefficient.
template <int STAGE> struct Fetch {
    double h, qx, qy, z;
    double ph, pqx, pqy, coef;
    double sy;  // sign applied to qy (wall ghost rows)
    int ys;     // ghost row of an imposed south (2) or north (3) side, else -1
};

// rh = d.rcp(c.h); the numerators are bounded by the caller (note_cell)
template <class D>
__host__ __device__ __forceinline__ Prim prim_x(const RawCell& c, double h_eps, const Recip& rh,
                                                D& d) {
    Prim p;
    p.h = c.h;
    if (c.h > h_eps) {
        p.un = d.div(c.qx, rh);
        p.ut = d.div(c.qy, rh);
    } else {
        p.un = 0.0;
        p.ut = 0.0;
    }
    p.eta = c.h + c.z;
    return p;
}

__host__ __device__ __forceinline__ Prim prim_x(const RawCell& c, double h_eps) {
    ExactDiv d;
    return prim_x(c, h_eps, d.rcp(c.h), d);
}

// The values of a cell that bound the operands of its quotients: depth,
// discharges, bed and velocities.
template <class D>
__device__ __forceinline__ void note_cell(D& d, const RawCell& r, const Prim& pr) {
    d.depth(r.h);
    d.cap(r.qx);
    d.cap(r.qy);
    d.low2(r.qx, r.qy);
    d.cap(r.z);
    d.cap(pr.un);
    d.cap(pr.ut);
    d.settle();
}

// y-view of a cell's primitives: normal velocity v, tangential u
__host__ __device__ __forceinline__ Prim to_y(const Prim& px) {
    Prim p;
    p.h = px.h;
    p.un = px.ut;
    p.ut = px.un;
    p.eta = px.eta;
    return p;
}

// Ghost of a side with an imposed depth or inflow discharge (Section 2.2:
// the ghost state from the Riemann invariants).  `o` holds the stage input
// of the boundary cell and becomes the ghost.  w is the outward normal
// velocity and c = sqrt(g h); the invariant w + 2c leaves the domain with
// the characteristic w + c and the ghost keeps it.  A boundary cell in
// supercritical outflow (w > c) keeps a free ghost (the copy).  Otherwise:
// depth imposed, the ghost's w from the invariant; inflow discharge q_b
// imposed, the ghost's depth h from 2 sqrt(g h) - q_b / h = w + 2c (increasing
// in h) by a fixed bisection; both imposed (supercritical inflow), the
// ghost is (h_b, q_b).  The tangential velocity is the cell's.  Every
// operation is a correctly rounded IEEE one (plain quotients and roots), so
// the ghost is reproducible bit for bit.
__device__ __forceinline__ RawCell imposed_ghost(const KParams& p, int side, RawCell o) {
    const bool xn = side < 2;
    const double sg = (side & 1) ? 1.0 : -1.0;  // outward normal: -x, +x, -y, +y
    const double hb = o.h;
    const double qo = sg * (xn ? o.qx : o.qy);
    const double qt = xn ? o.qy : o.qx;
    const bool wet = hb > p.h_eps;
    const double w = wet ? qo / hb : 0.0;
    const double vt = wet ? qt / hb : 0.0;
    const double c = sqrt(p.g * hb);
    if (w > c) return o;
    // constant indices only: a dynamic index into the kernel argument would
    // copy it to scratch memory
    const int type = side == 0 ? p.bcw : side == 1 ? p.bce : side == 2 ? p.bcs : p.bcn;
    const double hbc = side == 0   ? p.bc_h[0]
                       : side == 1 ? p.bc_h[1]
                       : side == 2 ? p.bc_h[2]
                                   : p.bc_h[3];
    const double qbc = side == 0   ? p.bc_q[0]
                       : side == 1 ? p.bc_q[1]
                       : side == 2 ? p.bc_q[2]
                                   : p.bc_q[3];
    double hg, qog;
    if (type == SWE_BC_IMPOSED_HQ) {
        hg = hbc;
        qog = -qbc;
    } else if (type == SWE_BC_IMPOSED_H) {
        hg = hbc;
        const double wg = (w + 2.0 * c) - 2.0 * sqrt(p.g * hg);
        qog = hg * wg;
    } else {
        const double qb = qbc;
        const double R = w + 2.0 * c;
        double hi = 1.0;
        for (int k = 0; k < 200 && 2.0 * sqrt(p.g * hi) - qb / hi < R; ++k) hi = 2.0 * hi;
        double lo = 0.0;
        for (int k = 0; k < 100; ++k) {
            const double mid = 0.5 * (lo + hi);
            if (2.0 * sqrt(p.g * mid) - qb / mid < R) lo = mid;
            else hi = mid;
        }
        hg = hi;
        qog = -qb;
    }
    const double qtg = hg * vt;
    o.h = hg;
    if (xn) {
        o.qx = sg * qog;
        o.qy = qtg;
    } else {
        o.qy = sg * qog;
        o.qx = qtg;
    }
    return o;
}

// The element at byte offset `off` of a row that starts at `row`.  In the
// tile kernels the row is the same for every lane of the block (scalar
// registers) and `off` is the lane's column times the element size, the
// same vector register for every array: each access is one load or store
// with a scalar base and a 32-bit vector offset, with no 64-bit address
// arithmetic per array.  Columns are below 2^28 (check_params), so the
// offset fits in 32 bits.
template <class T>
__device__ __forceinline__ T& at(T* row, uint32_t off) {
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return *reinterpret_cast<T*>(reinterpret_cast<B*>(row) + off);
}

// Issue the loads of cell (row r, mapped column at byte offset o).
template <int STAGE>
__device__ __forceinline__ Fetch<STAGE> fetch(const MemberArgs& m, const TileIO& io, int r,
                                              uint32_t o) {
    Fetch<STAGE> f;
    int rs = map_index(r, m.p.ny, m.p.bcs, m.p.bcn, f.sy);
    f.ys = (r < 0 && r >= -HALO && m.p.bcs >= SWE_BC_IMPOSED_H)                ? 2
           : (r >= m.p.ny && r < m.p.ny + HALO && m.p.bcn >= SWE_BC_IMPOSED_H) ? 3
                                                                               : -1;
    const size_t ro = (size_t)rs * m.p.nx;
    f.h = at(io.h + ro, o);
    f.qx = at(io.qx + ro, o);
    f.qy = at(io.qy + ro, o);
    f.z = at(m.z + ro, o);
    if (STAGE == 2) {
        f.ph = at(io.ph + ro, o);
        f.pqx = at(io.pqx + ro, o);
        f.pqy = at(io.pqy + ro, o);
        f.coef = m.fric ? at(m.fric + ro, o) : m.p.coef;
    } else {
        f.ph = f.pqx = f.pqy = f.coef = 0.0;
    }
    return f;
}

// Stage input of a fetched cell.  Stage 1: U^n.  Stage 2: U* =
// friction(U^n + dt Phi(U^n)) (the first stage of Heun's method, Section
// 3.2).  Ghost sign flips (walls) are applied last.
template <int STAGE, class D>
__device__ __forceinline__ RawCell build(const KParams& p, const Fetch<STAGE>& f, double sx,
                                         double dt, D& d) {
    RawCell o;
    o.z = f.z;
    if (STAGE == 1) {
        o.h = f.h;
        o.qx = f.qx;
        o.qy = f.qy;
    } else {
        double h1 = f.h + dt * f.ph;
        double qx1 = f.qx + dt * f.pqx;
        double qy1 = f.qy + dt * f.pqy;
        friction(p, f.coef, f.h, f.qx, f.qy, h1, qx1, qy1, dt, d);
        o.h = h1;
        o.qx = qx1;
        o.qy = qy1;
    }
    o.qx = sx * o.qx;
    o.qy = f.sy * o.qy;
    return o;
}

__device__ __forceinline__ unsigned long long as_bits(double x) {
    return (unsigned long long)__double_as_longlong(x);
}

// (Ax, Ay) of a step: the maximum over the accumulator pairs, reduced by
// the first AMAX_SPREAD lanes of each wave and broadcast to all lanes
__device__ __forceinline__ void read_amax(const unsigned long long* acc, double& ax, double& ay) {
    const int l = threadIdx.x & 63;
    unsigned long long x = 0ull, y = 0ull;
    if (l < AMAX_SPREAD) {
        x = acc[l * AMAX_LINE + 0];
        y = acc[l * AMAX_LINE + 1];
    }
    for (int off = AMAX_SPREAD / 2; off > 0; off >>= 1) {
        unsigned long long ox = __shfl_xor(x, off, 64);
        unsigned long long oy = __shfl_xor(y, off, 64);
        x = x < ox ? ox : x;
        y = y < oy ? oy : y;
    }
    x = __shfl(x, 0, 64);
    y = __shfl(y, 0, 64);
    ax = __longlong_as_double((long long)x);
    ay = __longlong_as_double((long long)y);
}

// block-wide maximum of two non-negative doubles, then one atomic each into
// accumulator pair `spread` mod AMAX_SPREAD of dst
template <int TXT>
__device__ void block_max2(double ax, double ay, unsigned long long* dst, int spread) {
    __shared__ double red[2][TXT / 64];
    for (int off = 32; off > 0; off >>= 1) {
        double ox = __shfl_down(ax, off, 64);
        double oy = __shfl_down(ay, off, 64);
        ax = ax < ox ? ox : ax;
        ay = ay < oy ? oy : ay;
    }
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = ax;
        red[1][wave] = ay;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mx = red[0][0], my = red[1][0];
        for (int w = 1; w < TXT / 64; ++w) {
            mx = mx < red[0][w] ? red[0][w] : mx;
            my = my < red[1][w] ? red[1][w] : my;
        }
        // non-negative doubles order like their bit patterns; NaN speeds
        // never enter the maximum (every comparison with NaN is false), as
        // in the oracle, and a non-finite state is flagged by the update
        unsigned long long* pair = dst + (spread & (AMAX_SPREAD - 1)) * AMAX_LINE;
        atomicMax(&pair[0], as_bits(mx));
        atomicMax(&pair[1], as_bits(my));
    }
}

// ---------------------------------------------------------------------------
// One tile through one stage
// ---------------------------------------------------------------------------

// Neighbour exchange inside one wave64 (tiles one wave wide): the value of
// lane t-1 (lane 0 keeps its own) and of lane t+1 (lane 63 keeps its own),
// moved by the full-wave DPP shifts.
__device__ __forceinline__ double from_left(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false);  // wave_shr:1
    hi = __builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_right(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false);  // wave_shl:1
    hi = __builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Stage 2: U^n of rows j, j+1 and j+2 of each lane's column (slot = row mod
// 3), kept from the row's fetch for Heun's average of row j; each lane reads
// and writes its own column only.  Stage 1 has none.
template <int TXT, int STAGE> struct UnRing {
    double v[3][3][TXT];
};
template <int TXT> struct UnRing<TXT, 1> {};

template <int TXT, int STAGE> struct TileLds {
    double h[2][TXT], u[2][TXT], v[2][TXT], e[2][TXT];  // primitives of row j (j & 1)
    double hm[TXT], zm[TXT], unm[TXT], utm[TXT];  // x-reconstruction, face i-1/2 side
    double f0[TXT], f1[TXT], f2[TXT];             // x-fluxes
    int bad[2];                                   // operand bounds broken in row j (j & 1)
    UnRing<TXT, STAGE> un;
};

// End of a step for a cell: rain R = r(t) w and Green-Ampt with the
// cell's soil (the optional fields are compiled in only for launches that
// have some), then U^{n+1} and V_inf written and the sticky flags raised.
// The cell is element ro of each array plus the byte offset o (see at()).
template <bool FIELDS>
__device__ __forceinline__ void finish_cell(const MemberArgs& m, const TileIO& io, size_t ro,
                                            uint32_t o, double dt, double rain, double hn,
                                            double qxn, double qyn, double vi) {
    const KParams& p = m.p;
    double rate = rain, gks = p.ks, gpsi = p.psi, gdth = p.dtheta;
    if constexpr (FIELDS) {
        if (m.rain_w) rate = rain * at(m.rain_w + ro, o);
        if (p.infil) {
            if (m.ks_f) gks = at(m.ks_f + ro, o);
            if (m.psi_f) gpsi = at(m.psi_f + ro, o);
            if (m.dth_f) gdth = at(m.dth_f + ro, o);
        }
    }
    rain_infiltration(p, dt, rate, gks, gpsi, gdth, hn, qxn, qyn, vi);
    // stored with the non-temporal hint: nothing reads them again before
    // the next step, and the caches are left to the rows a tile re-reads
    if (p.infil) __builtin_nontemporal_store(vi, &at(m.vinf + ro, o));
    __builtin_nontemporal_store(hn, &at(io.ho + ro, o));
    __builtin_nontemporal_store(qxn, &at(io.qxo + ro, o));
    __builtin_nontemporal_store(qyn, &at(io.qyo + ro, o));
    bool fin = (hn - hn) == 0.0 && (qxn - qxn) == 0.0 && (qyn - qyn) == 0.0;
    if (!fin)
        atomicOr(&m.sc->status, (unsigned)SWE_FLAG_NONFINITE);
    else if (hn < 0.0)
        atomicOr(&m.sc->status, (unsigned)SWE_FLAG_NEGDEPTH);
}

// March rows y0 .. y1-1 of a tile with division policy D (see Division).
// A tile one wave wide (TXT = 64) exchanges x-neighbours with DPP lane
// shifts and takes its decisions by a wave vote: no LDS, no barrier.  Wider
// tiles use LDS with two barriers per row: the primitives of row j+1 go to
// LDS (buffer (j+1) & 1) together with the x-fluxes of row j, before the
// second barrier of row j, so the reconstruction of row j+1 finds them there.
// With FastDiv a lane that finds its bounds broken in row j raises
// L.bad[j & 1] before the row's last barrier; every lane reads the flag
// after it and the march returns j before anything of row j is stored, for
// the caller to march on from row j with ExactDiv.  Thread 0 lowers the flag
// of row j+1 after the first barrier of row j, when every lane has read it
// for row j-1.  Returns y1 when the tile is done.

template <int STAGE, int TXT, class D, bool FIELDS, int ORDER, int FLUX, bool PHI2>
__device__ __forceinline__ int march(const MemberArgs& m, const TileIO& io, int strip, int y0,
                                     int y1, double dt, double rain, double& ax, double& ay,
                                     TileLds<TXT, STAGE>& L) {
    constexpr int OUTW = TXT - 2 * HALO;
    constexpr bool FAST = !std::is_same<D, ExactDiv>::value;
    const KParams& p = m.p;
    const int t = threadIdx.x;
    const int x0 = strip * OUTW;
    const int c = x0 - HALO + t;
    const bool out_col = (t >= HALO) && (t < TXT - HALO) && (c < p.nx);
    // byte offset of the output column (used by out_col lanes only)
    uint32_t oc = (uint32_t)c * (uint32_t)sizeof(double);
    const bool col_in = (c >= 0) && (c < p.nx);
    // a face c+1/2 computed by thread t has valid neighbour data when
    // 1 <= t <= TXT-3; it is a real face when -1 <= c <= nx-1
    const bool xface_ok = (t >= 1) && (t <= TXT - 3) && (c >= -1) && (c <= p.nx - 1);
    const int tl = t > 0 ? t - 1 : t;
    const int tr = t < TXT - 1 ? t + 1 : t;

    double sx;
    const int cs = map_index(c, p.nx, p.bcw, p.bce, sx);
    // byte offset of the mapped column (map_index keeps it inside the grid)
    uint32_t os = (uint32_t)cs * (uint32_t)sizeof(double);
    // x-ghost column of an imposed west (0) or east (1) side
    const int xside = !(FIELDS && p.imposed)                               ? -1
                      : (c < 0 && p.bcw >= SWE_BC_IMPOSED_H)               ? 0
                      : (c >= p.nx && c < p.nx + HALO && p.bce >= SWE_BC_IMPOSED_H) ? 1
                                                                                    : -1;
    D d;
    // stage input of a fetched cell, ghosts of imposed sides transformed
    auto cell = [&](const Fetch<STAGE>& f) {
        RawCell r = build<STAGE>(p, f, sx, dt, d);
        if (FIELDS) {
            const int side = xside >= 0 ? xside : (p.imposed ? f.ys : -1);
            if (side >= 0) r = imposed_ghost(p, side, r);
        }
        return r;
    };
    // X / dx and Y / dy: exact products when dx and dy are powers of two,
    // else quotients sharing the reciprocals of dx and dy
    const Recip Rdx = d.rcp(p.dx), Rdy = d.rcp(p.dy);

    // --- prologue: rows y0-2 .. y0+1, face y0-1/2; stage 1 prefetches row
    // y0+2 ------------------------------------------------------------------
    Fetch<STAGE> fA = fetch<STAGE>(m, io, y0 - 2, os);
    Fetch<STAGE> fB = fetch<STAGE>(m, io, y0 - 1, os);
    Fetch<STAGE> fC = fetch<STAGE>(m, io, y0, os);
    Fetch<STAGE> fD = fetch<STAGE>(m, io, y0 + 1, os);
    Fetch<STAGE> fnext;
    if (STAGE == 1) fnext = fetch<STAGE>(m, io, y0 + 2, os);
    RawCell rA = cell(fA);
    RawCell rB = cell(fB);
    RawCell rC = cell(fC);
    RawCell rD = cell(fD);
    // reciprocals of the depths of rows j and j+1, shared by the velocities
    // and by both reconstructions of the cell
    Recip R0 = d.rcp(rC.h), R1 = d.rcp(rD.h);
    Prim pA = prim_x(rA, p.h_eps, d.rcp(rA.h), d);
    Prim pB = prim_x(rB, p.h_eps, d.rcp(rB.h), d);
    Prim p0 = prim_x(rC, p.h_eps, R0, d), p1 = prim_x(rD, p.h_eps, R1, d);
    note_cell(d, rA, pA);
    note_cell(d, rB, pB);
    note_cell(d, rC, p0);
    note_cell(d, rD, p1);
    // stage input discharges of rows j and j+1 (stage 2 needs them for U**)
    double q0x = rC.qx, q0y = rC.qy, q1x = rD.qx, q1y = rD.qy;
    if constexpr (STAGE == 2) {
        // U^n of rows y0 and y0+1 for Heun's average
        const int s0 = y0 % 3, s1 = (y0 + 1) % 3;
        L.un.v[s0][0][t] = fC.h; L.un.v[s0][1][t] = fC.qx; L.un.v[s0][2][t] = fC.qy;
        L.un.v[s1][0][t] = fD.h; L.un.v[s1][1][t] = fD.qx; L.un.v[s1][2][t] = fD.qy;
    }

    Rec rprev = reconstruct<ORDER>(to_y(pA), to_y(pB), to_y(p0), p.h_eps, d.rcp(pB.h), d);
    Rec rcur = reconstruct<ORDER>(to_y(pB), to_y(p0), to_y(p1), p.h_eps, R0, d);
    // stage 2: the centred source of the y-reconstruction, taken when the
    // reconstruction is made, so that only its face j+1/2 side stays live
    double fcy_cur = STAGE == 2 ? centred(p.g, rcur) : 0.0;
    double gm0, gm1, gm2;  // face below the current row, as seen from above
    double gm_speed = 0.0;
    {
        FaceOut gm = face<FLUX>(p.g, rprev.h_p, rprev.z_p, rprev.un_p, rprev.ut_p, rcur.h_m,
                          rcur.z_m, rcur.un_m, rcur.ut_m, d);
        if (STAGE == 1 && y0 == 0)
            gm_speed = face_speed<FLUX>(p.g, rprev.h_p, rprev.un_p, rcur.h_m, rcur.un_m, d);
        gm0 = gm.f0;
        gm1 = gm.fr1;
        gm2 = gm.f2;
    }

    constexpr bool WAVE = TXT == 64;
    if (!WAVE) {
        // primitives of row y0 for the x-reconstruction of the first row
        L.h[y0 & 1][t] = p0.h;
        L.u[y0 & 1][t] = p0.un;
        L.v[y0 & 1][t] = p0.ut;
        L.e[y0 & 1][t] = p0.eta;
        if (FAST && t == 0) {
            L.bad[0] = 0;
            L.bad[1] = 0;
        }
        __syncthreads();
    }

    for (int j = y0; j < y1; ++j) {
        // The column offsets are opaque to the compiler from here: it cannot
        // fold them into each array's base before the loop (one 64-bit
        // address per array, live across the loop), so every access takes
        // its row in scalar registers and the offset as it is.
        asm volatile("" : "+v"(os), "+v"(oc));
        // Stage 1: the loads of row j+2 were issued one iteration ahead;
        // issue j+3.  Stage 2 issues those of row j+2 here and uses them
        // after the x direction of row j, which hides their latency and keeps
        // the two directions' temporaries from being live together (three
        // waves per SIMD instead of two).
        Fetch<STAGE> f2;
        if (STAGE == 2) {
            f2 = fetch<STAGE>(m, io, j + 2, os);
        } else {
            f2 = fnext;
            if (j + 1 < y1) fnext = fetch<STAGE>(m, io, j + 3, os);
        }

        // ---- y direction, all in registers ----
        RawCell r2;
        Recip R2;
        Prim p2;
        Rec rnext;
        FaceOut gp;
        double gp_speed = 0.0, fcy_next = 0.0;
        double Y0, Y1, Y2;
        auto y_direction = [&]() {
            if constexpr (STAGE == 2) {
                // U^n of row j+2, for its Heun average two rows later
                const int s2 = (j + 2) % 3;
                L.un.v[s2][0][t] = f2.h; L.un.v[s2][1][t] = f2.qx; L.un.v[s2][2][t] = f2.qy;
            }
            r2 = cell(f2);
            R2 = d.rcp(r2.h);
            p2 = prim_x(r2, p.h_eps, R2, d);
            note_cell(d, r2, p2);
            d.settle();
            rnext = reconstruct<ORDER>(to_y(p0), to_y(p1), to_y(p2), p.h_eps, R1, d);
            if (STAGE == 2) fcy_next = centred(p.g, rnext);
            gp = face<FLUX>(p.g, rcur.h_p, rcur.z_p, rcur.un_p, rcur.ut_p, rnext.h_m, rnext.z_m,
                            rnext.un_m, rnext.ut_m, d);
            if (STAGE == 1)
                gp_speed = face_speed<FLUX>(p.g, rcur.h_p, rcur.un_p, rnext.h_m, rnext.un_m, d);
            d.settle();
            const double fcy = STAGE == 2 ? fcy_cur : centred(p.g, rcur);
            Y0 = gp.f0 - gm0;
            Y1 = gp.fl1 - gm1 - fcy;  // normal momentum (qy)
            Y2 = gp.f2 - gm2;         // tangential momentum (qx)
        };
        if (STAGE == 1) y_direction();

        // ---- x direction, neighbours through DPP or LDS ----
        const int b = j & 1;
        Prim pl, pr;
        if (WAVE) {
            pl.h = from_left(p0.h); pl.un = from_left(p0.un);
            pl.ut = from_left(p0.ut); pl.eta = from_left(p0.eta);
            pr.h = from_right(p0.h); pr.un = from_right(p0.un);
            pr.ut = from_right(p0.ut); pr.eta = from_right(p0.eta);
        } else {
            pl.h = L.h[b][tl]; pl.un = L.u[b][tl]; pl.ut = L.v[b][tl]; pl.eta = L.e[b][tl];
            pr.h = L.h[b][tr]; pr.un = L.u[b][tr]; pr.ut = L.v[b][tr]; pr.eta = L.e[b][tr];
        }
        Rec rx = reconstruct<ORDER>(pl, p0, pr, p.h_eps, R0, d);
        double hm_r, zm_r, unm_r, utm_r;
        if (WAVE) {
            hm_r = from_right(rx.h_m);
            zm_r = from_right(rx.z_m);
            unm_r = from_right(rx.un_m);
            utm_r = from_right(rx.ut_m);
        } else {
            L.hm[t] = rx.h_m;
            L.zm[t] = rx.z_m;
            L.unm[t] = rx.un_m;
            L.utm[t] = rx.ut_m;
            __syncthreads();
            if (FAST && t == 0) L.bad[(j + 1) & 1] = 0;
            hm_r = L.hm[tr];
            zm_r = L.zm[tr];
            unm_r = L.unm[tr];
            utm_r = L.utm[tr];
        }
        FaceOut fp = face<FLUX>(p.g, rx.h_p, rx.z_p, rx.un_p, rx.ut_p, hm_r, zm_r, unm_r, utm_r, d);
        double fp_speed = 0.0;
        if (STAGE == 1) fp_speed = face_speed<FLUX>(p.g, rx.h_p, rx.un_p, hm_r, unm_r, d);
        d.settle();
        const double fcx = centred(p.g, rx);
        if (!WAVE) {
            L.f0[t] = fp.f0;
            L.f1[t] = fp.fr1;
            L.f2[t] = fp.f2;
            L.h[b ^ 1][t] = p1.h;
            L.u[b ^ 1][t] = p1.un;
            L.v[b ^ 1][t] = p1.ut;
            L.e[b ^ 1][t] = p1.eta;
        }
        // stage 2: the y direction, before the row's operand-bounds vote so
        // that the vote covers it
        if (STAGE == 2) y_direction();
        // stage 2: V_inf and the friction coefficient of the output row
        // (read again if it is a field), and its U^n for Heun's average from
        // the ring, rather than kept in registers since the row was fetched
        double vi = 0.0, n0h = 0.0, n0x = 0.0, n0y = 0.0, c0 = 0.0;
        if constexpr (STAGE == 2) {
            const int s0 = j % 3;
            n0h = L.un.v[s0][0][t];
            n0x = L.un.v[s0][1][t];
            n0y = L.un.v[s0][2][t];
            if (out_col) {
                if (p.infil) vi = at(m.vinf + (size_t)j * p.nx, oc);
                c0 = m.fric ? at(m.fric + (size_t)j * p.nx, oc) : p.coef;
            }
        }
        double fm0, fm1, fm2;
        if (WAVE) {
            if (FAST && __builtin_amdgcn_ballot_w64(!d.ok()) != 0) return j;
            fm0 = from_left(fp.f0);
            fm1 = from_left(fp.fr1);
            fm2 = from_left(fp.f2);
        } else {
            if (FAST && !d.ok()) L.bad[j & 1] = 1;
            __syncthreads();
            if (FAST && __builtin_amdgcn_readfirstlane(L.bad[j & 1]) != 0) return j;
            fm0 = L.f0[tl];
            fm1 = L.f1[tl];
            fm2 = L.f2[tl];
        }

        if (STAGE == 1) {
            if (j == 0 && col_in) ay = fmax(ay, gm_speed);
            if (col_in) ay = fmax(ay, gp_speed);
            if (xface_ok) ax = fmax(ax, fp_speed);
        }
        double X0 = fp.f0 - fm0;
        double X1 = fp.fl1 - fm1 - fcx;  // normal momentum (qx)
        double X2 = fp.f2 - fm2;         // tangential momentum (qy)

        if (out_col) {
            // the rest of the row is lane-local: with FastDiv a lane whose
            // bounds fail computes it again with IEEE division
            double rh, rqx, rqy;
            double h2 = 0.0, qx2 = 0.0, qy2 = 0.0;
            auto tail = [&](auto& dv) {
                if (p.dxy_pow2) {
                    rh = -(X0 * p.inv_dx + Y0 * p.inv_dy);
                    rqx = -(X1 * p.inv_dx + Y2 * p.inv_dy);
                    rqy = -(X2 * p.inv_dx + Y1 * p.inv_dy);
                } else {
                    // |X|, |Y| < 2^253 follow from the face bounds
                    dv.low2(X0, Y0);
                    dv.low2(X1, Y2);
                    dv.low2(X2, Y1);
                    rh = -(dv.div(X0, Rdx) + dv.div(Y0, Rdy));
                    rqx = -(dv.div(X1, Rdx) + dv.div(Y2, Rdy));
                    rqy = -(dv.div(X2, Rdx) + dv.div(Y1, Rdy));
                }
                if (STAGE == 2) {
                    // U** = friction(U* + dt Phi(U*)), stage input U*
                    h2 = p0.h + dt * rh;
                    qx2 = q0x + dt * rqx;
                    qy2 = q0y + dt * rqy;
                    friction(p, c0, p0.h, q0x, q0y, h2, qx2, qy2, dt, dv);
                }
            };
            if (FAST) {
                D lt;
                tail(lt);
                if (!lt.ok()) {
                    ExactDiv ed;
                    tail(ed);
                }
            } else {
                tail(d);
            }
            const size_t ro = (size_t)j * p.nx;
            if (STAGE == 1) {
                // the rate is read once, by stage 2: non-temporal hint
                __builtin_nontemporal_store(rh, &at(io.ph + ro, oc));
                __builtin_nontemporal_store(rqx, &at(io.pqx + ro, oc));
                __builtin_nontemporal_store(rqy, &at(io.pqy + ro, oc));
            } else {
                if constexpr (PHI2) {
                    at(io.ph2 + ro, oc) = rh;
                    at(io.pqx2 + ro, oc) = rqx;
                    at(io.pqy2 + ro, oc) = rqy;
                }
                // Heun: U^{n+1} = (U^n + U**)/2
                double hn = 0.5 * (n0h + h2);
                double qxn = 0.5 * (n0x + qx2);
                double qyn = 0.5 * (n0y + qy2);
                finish_cell<FIELDS>(m, io, ro, oc, dt, rain, hn, qxn, qyn, vi);
            }
        }

        // ---- shift the rolling window ----
        p0 = p1;
        p1 = p2;
        R0 = R1;
        R1 = R2;
        q0x = q1x; q0y = q1y;
        q1x = r2.qx; q1y = r2.qy;
        rcur = rnext;
        fcy_cur = fcy_next;
        gm0 = gp.f0;
        gm1 = gp.fr1;
        gm2 = gp.f2;
    }
    return y1;
}

// Rain intensity r(t) at the start time t of a step (rain is explicit,
// Section 3.1): the value of the last hyetograph breakpoint at or before t,
// 0 before the first, the parameters' constant without a hyetograph.  The
// breakpoints increase strictly, so those at or before t are a prefix of
// the table; each wave counts it with two ballots.
__device__ __forceinline__ double rain_rate(const MemberArgs& m, double t) {
    const int n = m.sc->hy_n;
    if (n <= 0) return m.p.rain;
    const int l = threadIdx.x & 63;
    const bool a = l < n && m.sc->hy_t[l] <= t;
    const bool b = l + 64 < n && m.sc->hy_t[l + 64] <= t;
    const int k = __popcll(__ballot(a)) + __popcll(__ballot(b));
    return k == 0 ? 0.0 : m.sc->hy_r[k - 1];
}

// Start of the update of a step: dt from the wave-speed bounds of stage 1
// (eq. cfl), the rain r(t) at the step's start time, and, by thread 0 of
// the lead block, the time, step count and dt log of the next slot.
// Returns false when no step is taken: dt not positive, not finite (raises
// the sticky DT flag) or below dt_min without being the step clipped to the
// end time (raises DT_UNDERFLOW; a frozen dt is taken as given).
__device__ __forceinline__ bool begin_step(const MemberArgs& m, const TileIO& io, bool lead,
                                           double& dt, double& rain) {
    double ax, ay;
    read_amax(&m.sc->amax[io.slot][0][0], ax, ay);
    double tc = m.sc->t[io.slot];
    rain = rain_rate(m, tc);
    const bool frozen = io.dt_fixed > 0.0;
    dt = frozen ? io.dt_fixed : time_step(m.p, ax, ay, tc, io.t_end);
    const bool finite = (dt - dt) == 0.0;  // false for inf and NaN
    const bool collapse = !frozen && dt < m.p.dt_min && dt < io.t_end - tc && dt > 0.0;
    const bool take = finite && dt > 0.0 && !collapse;
    if (lead && threadIdx.x == 0) {
        long long st = m.sc->steps[io.slot];
        if (take) {
            m.sc->t[io.slot ^ 1] = tc + dt;
            m.sc->steps[io.slot ^ 1] = st + 1;
            m.sc->last_dt = dt;
            m.sc->rain_depth += dt * rain;
            if (m.dtlog && st < m.dtlog_cap) m.dtlog[st] = dt;
        } else {
            m.sc->t[io.slot ^ 1] = tc;
            m.sc->steps[io.slot ^ 1] = st;
            if (!finite) atomicOr(&m.sc->status, (unsigned)SWE_FLAG_DT);
            if (collapse) atomicOr(&m.sc->status, (unsigned)SWE_FLAG_DT_UNDERFLOW);
        }
    }
    return take;
}

// First order (Section 3.3): the update of a step is one explicit Euler
// stage, U^{n+1} = friction(U^n + dt Phi(U^n)) (the convective and
// friction steps of Sections 3.1-3.2), then rain and Green-Ampt.  Cell by
// cell (no stencil): cells first, first + stride, ...
template <bool FIELDS>
__device__ __forceinline__ void euler_cells(const MemberArgs& m, const TileIO& io, bool lead,
                                            size_t first, size_t stride) {
    const KParams& p = m.p;
    const size_t n = (size_t)p.nx * (size_t)p.ny;
    double dt, rain;
    if (!begin_step(m, io, lead, dt, rain)) {
        for (size_t i = first; i < n; i += stride) {
            io.ho[i] = io.h[i];
            io.qxo[i] = io.qx[i];
            io.qyo[i] = io.qy[i];
        }
        return;
    }
    for (size_t i = first; i < n; i += stride) {
        const double h0 = io.h[i], qx0 = io.qx[i], qy0 = io.qy[i];
        double h1 = h0 + dt * io.ph[i];
        double qx1 = qx0 + dt * io.pqx[i];
        double qy1 = qy0 + dt * io.pqy[i];
        const double coef = m.fric ? m.fric[i] : p.coef;
        friction(p, coef, h0, qx0, qy0, h1, qx1, qy1, dt);
        const double vi = p.infil ? m.vinf[i] : 0.0;
        finish_cell<FIELDS>(m, io, i, 0u, dt, rain, h1, qx1, qy1, vi);
    }
}

// Whether a simulation has any optional per-cell rain or soil field (its
// stage-2 launches then take the FIELDS variant of the tile routine, as do
// both stages of a simulation with an imposed side).
__host__ __device__ __forceinline__ bool has_fields(const MemberArgs& m) {
    return m.rain_w || m.ks_f || m.psi_f || m.dth_f;
}

// STAGE 1 (rate): Phi(U^n) to io.ph/pqx/pqy and the face wave-speed bounds
// of eq. (cfl) into io.acc.  STAGE 2 (update): dt from the bounds, U* rebuilt
// on the fly, Phi(U*), U** = friction(U* + dt Phi(U*)), Heun's average,
// rain and Green-Ampt, U^{n+1} to io.ho/qxo/qyo.  `lead` marks the one tile
// per simulation that does the scalar bookkeeping (time, step count, dt log,
// clearing the next step's accumulators).
// `spread` picks the accumulator pair of stage 1 (any block-dependent index).
// FIELDS compiles in the reads of the optional rain and soil fields and the
// ghosts of imposed sides (imposed_ghost, when KParams::imposed); ORDER 1
// (stage 1 only) replaces MUSCL by the cell values (first order); FLUX 1
// takes the Rusanov flux instead of HLL, FLUX 2 the kinetic flux; PHI2
// (stage 2) also writes Phi(U*) to io.ph2/pqx2/pqy2 (the adjoint keeps it).
template <int STAGE, int TXT, bool FIELDS = false, int ORDER = 2, int FLUX = 0,
          bool PHI2 = false>
__device__ __forceinline__ void stage_tile(const MemberArgs& m, const TileIO& io, int strip,
                                           int y0, int y1, bool lead, int spread) {
    constexpr int OUTW = TXT - 2 * HALO;
    const KParams& p = m.p;
    const int t = threadIdx.x;
    const int c = strip * OUTW - HALO + t;
    const bool out_col = (t >= HALO) && (t < TXT - HALO) && (c < p.nx);

    __shared__ TileLds<TXT, STAGE> L;

    double dt = 0.0, rain = 0.0;
    if (STAGE == 2) {
        if (!begin_step(m, io, lead, dt, rain)) {
            // no step: U^{n+1} = U^n
            if (out_col) {
                for (int j = y0; j < y1; ++j) {
                    size_t idx = (size_t)j * p.nx + c;
                    io.ho[idx] = io.h[idx];
                    io.qxo[idx] = io.qx[idx];
                    io.qyo[idx] = io.qy[idx];
                }
            }
            return;
        }
    } else {
        if (io.clr && lead && t < AMAX_SPREAD) {
            io.clr[t * AMAX_LINE + 0] = 0ull;
            io.clr[t * AMAX_LINE + 1] = 0ull;
        }
    }

    double ax = 0.0, ay = 0.0;
    int stop = y0;
    if (p.fast_div)
        stop = march<STAGE, TXT, FastDiv, FIELDS, ORDER, FLUX, PHI2>(m, io, strip, y0, y1, dt,
                                                                     rain, ax, ay, L);
    if (stop < y1)
        march<STAGE, TXT, ExactDiv, FIELDS, ORDER, FLUX, PHI2>(m, io, strip, stop, y1, dt, rain,
                                                               ax, ay, L);
    if (STAGE == 1) block_max2<TXT>(ax, ay, io.acc, spread);
}

}  // namespace swe_dev
