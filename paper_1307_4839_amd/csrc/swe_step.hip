// HIP kernels and C ABI of the well-balanced 2D Saint-Venant step for
// MI355X (gfx950).
//
// Method: arXiv:1307.4839, Sections 2-3 (see include/swe.h for the map of
// formulas to sections).  One time step is two launches:
//
//   rate kernel   (stage 1): reads U^n and z, computes the convective rate
//                 Phi(U^n) of eq. (SW1Dscheme) extended to 2D by the method
//                 of lines, writes Phi (3 doubles per cell) and reduces the
//                 face wave-speed bounds Ax, Ay of eq. (cfl) with an
//                 atomic maximum.
//   update kernel (stage 2): every block derives the same dt from (Ax, Ay),
//                 rebuilds U* = friction(U^n + dt Phi(U^n)) on the fly for
//                 the cells of its window (Section 3.2), evaluates
//                 Phi(U*), forms U** = friction(U* + dt Phi(U*)), Heun's
//                 average (U^n + U**)/2, then rain and Green-Ampt
//                 infiltration (Section 3.5), and writes U^{n+1}.
//
// HBM traffic per cell and step: stage 1 reads 32 B and writes 24 B; stage 2
// reads 56 B (+8 B with a friction field, +8 B V_inf) and writes 24 B
// (+8 B V_inf).  Face values never go to HBM.
//
// Tiling: a block of 256 threads owns a strip of 256 columns, of which the
// 252 interior ones are outputs (two halo columns per side feed the
// second-order stencil), and marches down a segment of rows.  Along y the
// stencil lives in registers (each thread keeps a rolling window of its own
// column), so every y-face is evaluated once.  Along x neighbours exchange
// values through LDS, so every x-face is also evaluated once.  Boundary
// ghost cells (Section 2.2, two layers at second order, Section 6.1) are
// produced by index mapping in the loader; no ghost arrays exist in HBM.
//
// Arithmetic follows the formulas in the order they are written in the
// paper; with -ffp-contract=off and IEEE division and square root the only
// operation that is not correctly rounded is the cube root of the Manning
// law.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>

#include "swe.h"

namespace {

constexpr int TX = 256;                 // threads per block = strip width
constexpr int HALO = 2;                 // ghost/halo width at second order
constexpr int OUT_W = TX - 2 * HALO;    // output columns per strip
constexpr int DIAG_BLOCKS = 512;        // blocks of the diagnostics reduction

// ---------------------------------------------------------------------------
// Device-side scalars (in the workspace)
// ---------------------------------------------------------------------------

struct DevScalars {
    unsigned long long amax[3][2];  // per slot: bit patterns of Ax, Ay >= 0
    double t[2];                    // time, double-buffered by step parity
    long long steps[2];             // steps taken, double-buffered
    double last_dt;
    unsigned int status;            // sticky SWE_FLAG_* bits
    unsigned int pad;
};
static_assert(sizeof(DevScalars) <= 256, "scalar block must fit 256 bytes");

struct KParams {
    int nx, ny;
    double dx, dy, g, cfl, dt_max, h_eps;
    int bcw, bce, bcs, bcn;
    int law;
    double coef;
    double rain;
    int infil;
    double ks, psi, dtheta;
};

// ---------------------------------------------------------------------------
// Formulas (Sections 3.1, 3.3, 3.4)
// ---------------------------------------------------------------------------

// For ordered (non-NaN) operands these return the same value as the
// comparisons they replace (up to the sign of a zero, which no later
// operation can turn into a different non-zero value).
__device__ __forceinline__ double vmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return fmin(a, b); }

// minmod limiter, Section 3.4: min(a, b) if both >= 0, max(a, b) if both
// <= 0, else 0.  Branch-free form with the same value:
// max(min(a, b), min(max(a, b), 0)).
__device__ __forceinline__ double minmod(double a, double b) {
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
__device__ __forceinline__ Rec muscl(const Prim& a, const Prim& c, const Prim& b,
                                     double h_eps) {
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
        double wp = r.h_p / c.h;
        double wm = r.h_m / c.h;
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

// Flux through one face: hydrostatic reconstruction (Section 3.1), HLL
// (Section 3.3), and the normal-momentum corrections S_L (left cell) and
// S_R (right cell).  fl = flux seen by the left cell, fr = by the right one.
// speed = max(|u-| + sqrt(g h-), |u+| + sqrt(g h+)) on the MUSCL states.
struct FaceOut {
    double f0, fl1, fr1, f2;
    double speed;
};

__device__ __forceinline__ FaceOut face(double g, double hm, double zm, double unm,
                                        double utm, double hp, double zp, double unp,
                                        double utp) {
    double zs = vmax(zm, zp);
    double hL = vmax(hm + zm - zs, 0.0);
    double hR = vmax(hp + zp - zs, 0.0);
    double cL = sqrt(g * hL);
    double cR = sqrt(g * hR);
    double c1 = vmin(unm - cL, unp - cR);
    double c2 = vmax(unm + cL, unp + cR);
    double qL = hL * unm;
    double qR = hR * unp;
    double hg = 0.5 * g;
    double FL0 = qL, FL1 = qL * unm + hg * hL * hL, FL2 = qL * utm;
    double FR0 = qR, FR1 = qR * unp + hg * hR * hR, FR2 = qR * utp;
    double F0, F1, F2;
    if (0.0 <= c1) {
        F0 = FL0; F1 = FL1; F2 = FL2;
    } else if (c2 <= 0.0) {
        F0 = FR0; F1 = FR1; F2 = FR2;
    } else {
        double den = c2 - c1;
        double w = c1 * c2 / den;
        F0 = (c2 * FL0 - c1 * FR0) / den + w * (hR - hL);
        F1 = (c2 * FL1 - c1 * FR1) / den + w * (qR - qL);
        F2 = (c2 * FL2 - c1 * FR2) / den + w * (hR * utp - hL * utm);
    }
    double sL = hg * (hm * hm - hL * hL);
    double sR = hg * (hp * hp - hR * hR);
    FaceOut o;
    o.f0 = F0;
    o.fl1 = F1 + sL;
    o.fr1 = F1 + sR;
    o.f2 = F2;
    double sm = fabs(unm) + sqrt(g * hm);
    double sp = fabs(unp) + sqrt(g * hp);
    o.speed = fmax(sm, sp);
    return o;
}

// centred source Fc of Section 3.1 (normal momentum)
__device__ __forceinline__ double centred(double g, const Rec& r) {
    return (-g) * (0.5 * (r.h_m + r.h_p)) * (r.z_p - r.z_m);
}

// Semi-implicit friction of one stage (Section 3.2).  (h0, q0) stage input,
// (h1, q1) convective output.
__device__ __forceinline__ void friction(const KParams& p, double coef, double h0,
                                         double qx0, double qy0, double h1,
                                         double& qx1, double& qy1, double dt) {
    if (h1 <= p.h_eps) {
        qx1 = 0.0;
        qy1 = 0.0;
        return;
    }
    if (p.law == SWE_FRIC_NONE || !(h0 > p.h_eps)) return;
    double qn = sqrt(qx0 * qx0 + qy0 * qy0);
    double den;
    if (p.law == SWE_FRIC_DARCY)
        den = 1.0 + dt * (coef / 8.0) * qn / (h0 * h1);
    else
        den = 1.0 + dt * p.g * coef * coef * qn / (h0 * (h1 * cbrt(h1)));
    qx1 = qx1 / den;
    qy1 = qy1 / den;
}

// dt from the wave-speed bounds (eq. cfl in 2D), clipped to dt_max and to
// the remaining time.
__device__ __forceinline__ double time_step(const KParams& p, double ax, double ay,
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

// Rain, then Green-Ampt (Section 3.5); the infiltrated water leaves with the
// cell's velocity.
__device__ __forceinline__ void rain_infiltration(const KParams& p, double dt,
                                                  double& h, double& qx, double& qy,
                                                  double& vinf) {
    h = h + dt * p.rain;
    if (!p.infil) return;
    double d;
    if (vinf > 0.0) {
        double zf = vinf / p.dtheta;
        double ic = p.ks * (1.0 + (p.psi + h) / zf);
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

__device__ __forceinline__ int map_index(int c, int n, int bc_lo, int bc_hi,
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
// Kernel arguments
// ---------------------------------------------------------------------------

struct StageArgs {
    KParams p;
    int ty;                      // rows per block
    const double* h;             // U^n
    const double* qx;
    const double* qy;
    const double* z;
    const double* fric;          // per-cell coefficient or nullptr
    // stage 1 outputs / stage 2 inputs
    double* ph;
    double* pqx;
    double* pqy;
    // stage 2 outputs
    double* ho;
    double* qxo;
    double* qyo;
    double* vinf;
    DevScalars* sc;
    int slot;                    // step parity: amax slot and time buffer
    unsigned long long* amax_acc;    // stage 1: where (Ax, Ay) accumulate
    unsigned long long* amax_clear;  // stage 1: pair zeroed for the next step
    double t_end;
    double* dtlog;
    long long dtlog_cap;
};

struct RawCell {
    double h, qx, qy, z;
};

// Raw values of one cell of the stage input as read from HBM.  Stage 1:
// U^n and z.  Stage 2 also: Phi(U^n) and the friction coefficient.
template <int STAGE> struct Fetch {
    double h, qx, qy, z;
    double ph, pqx, pqy, coef;
    double sy;  // sign applied to qy (wall ghost rows)
};

__device__ __forceinline__ Prim prim_x(const RawCell& c, double h_eps) {
    Prim p;
    p.h = c.h;
    if (c.h > h_eps) {
        p.un = c.qx / c.h;
        p.ut = c.qy / c.h;
    } else {
        p.un = 0.0;
        p.ut = 0.0;
    }
    p.eta = c.h + c.z;
    return p;
}

// y-view of a cell's primitives: normal velocity v, tangential u
__device__ __forceinline__ Prim to_y(const Prim& px) {
    Prim p;
    p.h = px.h;
    p.un = px.ut;
    p.ut = px.un;
    p.eta = px.eta;
    return p;
}

// Issue the loads of cell (row r, mapped column cs).
template <int STAGE>
__device__ __forceinline__ Fetch<STAGE> fetch(const StageArgs& a, int r, int cs) {
    Fetch<STAGE> f;
    int rs = map_index(r, a.p.ny, a.p.bcs, a.p.bcn, f.sy);
    size_t idx = (size_t)rs * a.p.nx + cs;
    f.h = a.h[idx];
    f.qx = a.qx[idx];
    f.qy = a.qy[idx];
    f.z = a.z[idx];
    if (STAGE == 2) {
        f.ph = a.ph[idx];
        f.pqx = a.pqx[idx];
        f.pqy = a.pqy[idx];
        f.coef = a.fric ? a.fric[idx] : a.p.coef;
    } else {
        f.ph = f.pqx = f.pqy = f.coef = 0.0;
    }
    return f;
}

// Stage input of a fetched cell.  Stage 1: U^n.  Stage 2: U* =
// friction(U^n + dt Phi(U^n)) (the first stage of Heun's method, Section
// 3.2).  Ghost sign flips (walls) are applied last.
template <int STAGE>
__device__ __forceinline__ RawCell build(const KParams& p, const Fetch<STAGE>& f,
                                         double sx, double dt) {
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
        friction(p, f.coef, f.h, f.qx, f.qy, h1, qx1, qy1, dt);
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

// block-wide maximum of two non-negative doubles, then one atomic each
__device__ void block_max2(double ax, double ay, unsigned long long* dst) {
    __shared__ double red[2][TX / 64];
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
        for (int w = 1; w < TX / 64; ++w) {
            mx = mx < red[0][w] ? red[0][w] : mx;
            my = my < red[1][w] ? red[1][w] : my;
        }
        // non-negative doubles order like their bit patterns; NaN speeds
        // never enter the maximum (every comparison with NaN is false), as
        // in the oracle, and a non-finite state is flagged by the update
        atomicMax(&dst[0], as_bits(mx));
        atomicMax(&dst[1], as_bits(my));
    }
}

// ---------------------------------------------------------------------------
// The stage kernel (STAGE 1: rate; STAGE 2: update)
// ---------------------------------------------------------------------------

#ifndef SWE_STAGE_WAVES
#define SWE_STAGE_WAVES 1
#endif

template <int STAGE>
__global__ __launch_bounds__(TX) __attribute__((amdgpu_waves_per_eu(SWE_STAGE_WAVES)))
void stage_kernel(StageArgs a) {
    const KParams& p = a.p;
    const int t = threadIdx.x;
    const int x0 = blockIdx.x * OUT_W;
    const int c = x0 - HALO + t;
    const int y0 = blockIdx.y * a.ty;
    const int y1 = min(y0 + a.ty, p.ny);
    const bool out_col = (t >= HALO) && (t < TX - HALO) && (c < p.nx);
    const bool col_in = (c >= 0) && (c < p.nx);
    // a face c+1/2 computed by thread t has valid neighbour data when
    // 1 <= t <= TX-3; it is a real face when -1 <= c <= nx-1
    const bool xface_ok = (t >= 1) && (t <= TX - 3) && (c >= -1) && (c <= p.nx - 1);

    __shared__ double s_h[TX], s_u[TX], s_v[TX], s_e[TX];
    __shared__ double s_hm[TX], s_zm[TX], s_unm[TX], s_utm[TX];
    __shared__ double s_f0[TX], s_f1[TX], s_f2[TX];

    double dt = 0.0;
    if (STAGE == 2) {
        double ax = __longlong_as_double((long long)a.sc->amax[a.slot][0]);
        double ay = __longlong_as_double((long long)a.sc->amax[a.slot][1]);
        double tc = a.sc->t[a.slot];
        dt = time_step(p, ax, ay, tc, a.t_end);
        const bool finite = (dt - dt) == 0.0;  // false for inf and NaN
        if (blockIdx.x == 0 && blockIdx.y == 0 && t == 0) {
            long long st = a.sc->steps[a.slot];
            if (finite && dt > 0.0) {
                a.sc->t[a.slot ^ 1] = tc + dt;
                a.sc->steps[a.slot ^ 1] = st + 1;
                a.sc->last_dt = dt;
                if (a.dtlog && st < a.dtlog_cap) a.dtlog[st] = dt;
            } else {
                a.sc->t[a.slot ^ 1] = tc;
                a.sc->steps[a.slot ^ 1] = st;
                if (!finite) atomicOr(&a.sc->status, (unsigned)SWE_FLAG_DT);
            }
        }
        if (!(finite && dt > 0.0)) {
            // no step: U^{n+1} = U^n
            if (out_col) {
                for (int j = y0; j < y1; ++j) {
                    size_t idx = (size_t)j * p.nx + c;
                    a.ho[idx] = a.h[idx];
                    a.qxo[idx] = a.qx[idx];
                    a.qyo[idx] = a.qy[idx];
                }
            }
            return;
        }
    } else {
        if (a.amax_clear && blockIdx.x == 0 && blockIdx.y == 0 && t == 0) {
            a.amax_clear[0] = 0ull;
            a.amax_clear[1] = 0ull;
        }
    }

    double sx;
    const int cs = map_index(c, p.nx, p.bcw, p.bce, sx);

    // --- prologue: rows y0-2 .. y0+1, face y0-1/2; prefetch row y0+2 -------
    Fetch<STAGE> fA = fetch<STAGE>(a, y0 - 2, cs);
    Fetch<STAGE> fB = fetch<STAGE>(a, y0 - 1, cs);
    Fetch<STAGE> fC = fetch<STAGE>(a, y0, cs);
    Fetch<STAGE> fD = fetch<STAGE>(a, y0 + 1, cs);
    Fetch<STAGE> fnext = fetch<STAGE>(a, y0 + 2, cs);
    RawCell rC = build<STAGE>(p, fC, sx, dt);
    RawCell rD = build<STAGE>(p, fD, sx, dt);
    Prim pA = prim_x(build<STAGE>(p, fA, sx, dt), p.h_eps);
    Prim pB = prim_x(build<STAGE>(p, fB, sx, dt), p.h_eps);
    Prim p0 = prim_x(rC, p.h_eps), p1 = prim_x(rD, p.h_eps);
    // stage input discharges of rows j and j+1 (stage 2 needs them for U**)
    double q0x = rC.qx, q0y = rC.qy, q1x = rD.qx, q1y = rD.qy;
    // U^n of rows j and j+1 (stage 2: Heun's average)
    double n0h = fC.h, n0x = fC.qx, n0y = fC.qy, n1h = fD.h, n1x = fD.qx, n1y = fD.qy;
    double c0 = fC.coef, c1 = fD.coef;

    Rec rprev = muscl(to_y(pA), to_y(pB), to_y(p0), p.h_eps);
    Rec rcur = muscl(to_y(pB), to_y(p0), to_y(p1), p.h_eps);
    double ax = 0.0, ay = 0.0;
    double gm0, gm1, gm2;  // face below the current row, as seen from above
    {
        FaceOut gm = face(p.g, rprev.h_p, rprev.z_p, rprev.un_p, rprev.ut_p, rcur.h_m,
                          rcur.z_m, rcur.un_m, rcur.ut_m);
        if (y0 == 0 && col_in) ay = gm.speed;
        gm0 = gm.f0;
        gm1 = gm.fr1;
        gm2 = gm.f2;
    }

    for (int j = y0; j < y1; ++j) {
        // the loads of row j+2 were issued one iteration ahead; issue j+3
        Fetch<STAGE> f2 = fnext;
        if (j + 1 < y1) fnext = fetch<STAGE>(a, j + 3, cs);

        // ---- y direction, all in registers ----
        RawCell r2 = build<STAGE>(p, f2, sx, dt);
        Prim p2 = prim_x(r2, p.h_eps);
        Rec rnext = muscl(to_y(p0), to_y(p1), to_y(p2), p.h_eps);
        FaceOut gp = face(p.g, rcur.h_p, rcur.z_p, rcur.un_p, rcur.ut_p, rnext.h_m,
                          rnext.z_m, rnext.un_m, rnext.ut_m);
        if (STAGE == 1 && col_in) ay = fmax(ay, gp.speed);
        double fcy = centred(p.g, rcur);
        double Y0 = gp.f0 - gm0;
        double Y1 = gp.fl1 - gm1 - fcy;  // normal momentum (qy)
        double Y2 = gp.f2 - gm2;         // tangential momentum (qx)

        // ---- x direction, neighbours through LDS ----
        s_h[t] = p0.h;
        s_u[t] = p0.un;
        s_v[t] = p0.ut;
        s_e[t] = p0.eta;
        __syncthreads();
        Prim pl, pr;
        {
            int tl = t > 0 ? t - 1 : t;
            int tr = t < TX - 1 ? t + 1 : t;
            pl.h = s_h[tl]; pl.un = s_u[tl]; pl.ut = s_v[tl]; pl.eta = s_e[tl];
            pr.h = s_h[tr]; pr.un = s_u[tr]; pr.ut = s_v[tr]; pr.eta = s_e[tr];
        }
        Rec rx = muscl(pl, p0, pr, p.h_eps);
        s_hm[t] = rx.h_m;
        s_zm[t] = rx.z_m;
        s_unm[t] = rx.un_m;
        s_utm[t] = rx.ut_m;
        __syncthreads();
        FaceOut fp;
        {
            int tr = t < TX - 1 ? t + 1 : t;
            fp = face(p.g, rx.h_p, rx.z_p, rx.un_p, rx.ut_p, s_hm[tr], s_zm[tr],
                      s_unm[tr], s_utm[tr]);
        }
        if (STAGE == 1 && xface_ok) ax = fmax(ax, fp.speed);
        s_f0[t] = fp.f0;
        s_f1[t] = fp.fr1;
        s_f2[t] = fp.f2;
        __syncthreads();
        double fm0, fm1, fm2;
        {
            int tl = t > 0 ? t - 1 : t;
            fm0 = s_f0[tl];
            fm1 = s_f1[tl];
            fm2 = s_f2[tl];
        }
        double fcx = centred(p.g, rx);
        double X0 = fp.f0 - fm0;
        double X1 = fp.fl1 - fm1 - fcx;  // normal momentum (qx)
        double X2 = fp.f2 - fm2;         // tangential momentum (qy)

        double rh = -(X0 / p.dx + Y0 / p.dy);
        double rqx = -(X1 / p.dx + Y2 / p.dy);
        double rqy = -(X2 / p.dx + Y1 / p.dy);

        if (out_col) {
            size_t idx = (size_t)j * p.nx + c;
            if (STAGE == 1) {
                a.ph[idx] = rh;
                a.pqx[idx] = rqx;
                a.pqy[idx] = rqy;
            } else {
                // U** = friction(U* + dt Phi(U*)), stage input U*
                double h2 = p0.h + dt * rh;
                double qx2 = q0x + dt * rqx;
                double qy2 = q0y + dt * rqy;
                friction(p, c0, p0.h, q0x, q0y, h2, qx2, qy2, dt);
                // Heun: U^{n+1} = (U^n + U**)/2
                double hn = 0.5 * (n0h + h2);
                double qxn = 0.5 * (n0x + qx2);
                double qyn = 0.5 * (n0y + qy2);
                double vi = 0.0;
                if (p.infil) vi = a.vinf[idx];
                rain_infiltration(p, dt, hn, qxn, qyn, vi);
                if (p.infil) a.vinf[idx] = vi;
                a.ho[idx] = hn;
                a.qxo[idx] = qxn;
                a.qyo[idx] = qyn;
                bool fin = (hn - hn) == 0.0 && (qxn - qxn) == 0.0 && (qyn - qyn) == 0.0;
                if (!fin)
                    atomicOr(&a.sc->status, (unsigned)SWE_FLAG_NONFINITE);
                else if (hn < 0.0)
                    atomicOr(&a.sc->status, (unsigned)SWE_FLAG_NEGDEPTH);
            }
        }

        // ---- shift the rolling window ----
        p0 = p1;
        p1 = p2;
        q0x = q1x; q0y = q1y;
        q1x = r2.qx; q1y = r2.qy;
        n0h = n1h; n0x = n1x; n0y = n1y;
        n1h = f2.h; n1x = f2.qx; n1y = f2.qy;
        c0 = c1;
        c1 = f2.coef;
        rcur = rnext;
        gm0 = gp.f0;
        gm1 = gp.fr1;
        gm2 = gp.f2;
    }

    if (STAGE == 1) block_max2(ax, ay, a.amax_acc);
}

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------

__global__ void init_scalars_kernel(DevScalars* sc, double t) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        for (int s = 0; s < 3; ++s) {
            sc->amax[s][0] = 0ull;
            sc->amax[s][1] = 0ull;
        }
        sc->t[0] = t;
        sc->t[1] = t;
        sc->steps[0] = 0;
        sc->steps[1] = 0;
        sc->last_dt = 0.0;
        sc->status = 0u;
    }
}

__global__ void set_time_kernel(DevScalars* sc, int slot, double t) {
    if (threadIdx.x == 0 && blockIdx.x == 0) sc->t[slot] = t;
}

__global__ void clear_amax_kernel(DevScalars* sc, int slot) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc->amax[slot][0] = 0ull;
        sc->amax[slot][1] = 0ull;
    }
}

__global__ void copy3_kernel(const double* __restrict__ a, const double* __restrict__ b,
                             const double* __restrict__ c, double* __restrict__ A,
                             double* __restrict__ B, double* __restrict__ Cc, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        A[i] = a[i];
        B[i] = b[i];
        Cc[i] = c[i];
    }
}

// Deterministic diagnostics: block b reduces the cells b, b + B, b + 2B, ...
// in a fixed tree; a single block then combines the partials in order.
constexpr int DIAG_T = 256;

__global__ __launch_bounds__(DIAG_T) void diag_partial_kernel(
    const double* __restrict__ h, const double* __restrict__ vinf, double h_eps,
    size_t n, double* __restrict__ part) {
    __shared__ double s_m[DIAG_T], s_v[DIAG_T], s_lo[DIAG_T], s_hi[DIAG_T], s_w[DIAG_T];
    double m = 0.0, v = 0.0, lo = INFINITY, hi = -INFINITY, w = 0.0;
    for (size_t i = (size_t)blockIdx.x * DIAG_T + threadIdx.x; i < n;
         i += (size_t)gridDim.x * DIAG_T) {
        double x = h[i];
        m += x;
        if (vinf) v += vinf[i];
        lo = fmin(lo, x);
        hi = fmax(hi, x);
        if (x > h_eps) w += 1.0;
    }
    int t = threadIdx.x;
    s_m[t] = m; s_v[t] = v; s_lo[t] = lo; s_hi[t] = hi; s_w[t] = w;
    __syncthreads();
    for (int off = DIAG_T / 2; off > 0; off >>= 1) {
        if (t < off) {
            s_m[t] += s_m[t + off];
            s_v[t] += s_v[t + off];
            s_lo[t] = fmin(s_lo[t], s_lo[t + off]);
            s_hi[t] = fmax(s_hi[t], s_hi[t + off]);
            s_w[t] += s_w[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        double* o = part + (size_t)blockIdx.x * 5;
        o[0] = s_m[0]; o[1] = s_v[0]; o[2] = s_lo[0]; o[3] = s_hi[0]; o[4] = s_w[0];
    }
}

__global__ void diag_final_kernel(double* part, int nb) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double m = 0.0, v = 0.0, lo = INFINITY, hi = -INFINITY, w = 0.0;
        for (int b = 0; b < nb; ++b) {
            const double* o = part + (size_t)b * 5;
            m += o[0]; v += o[1]; lo = fmin(lo, o[2]); hi = fmax(hi, o[3]); w += o[4];
        }
        part[0] = m; part[1] = v; part[2] = lo; part[3] = hi; part[4] = w;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host runtime and C ABI
// ---------------------------------------------------------------------------

struct swe_ctx {
    swe_params prm;
    KParams kp;
    swe_buffers buf;
    hipStream_t stream;
    // workspace carve-up
    double* bh;   // second state
    double* bqx;
    double* bqy;
    double* ph;   // stage rate
    double* pqx;
    double* pqy;
    double* diag; // diagnostics partials
    DevScalars* sc;
    int slot;     // parity of the next step
    int ty;       // rows per block
    double* dtlog;
    long long dtlog_cap;
    // optional per-kernel timing: events before stage 1, between the
    // stages and after stage 2 of each profiled step
    hipEvent_t* prof_ev;
    int prof_cap;
    int prof_n;
};

namespace {

size_t ncells(const swe_params* p) { return (size_t)p->nx * (size_t)p->ny; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int check_params(const swe_params* p) {
    if (!p) return SWE_EINVAL;
    if (p->nx < 2 || p->ny < 2) return SWE_EINVAL;
    if (!(p->dx > 0.0) || !(p->dy > 0.0) || !(p->g > 0.0) || !(p->cfl > 0.0))
        return SWE_EINVAL;
    if (!(p->h_eps >= 0.0) || !(p->dt_max > 0.0)) return SWE_EINVAL;
    for (int k = 0; k < 4; ++k)
        if (p->bc[k] != SWE_BC_WALL && p->bc[k] != SWE_BC_OUTFLOW) return SWE_EINVAL;
    if (p->fric_law < SWE_FRIC_NONE || p->fric_law > SWE_FRIC_DARCY) return SWE_EINVAL;
    if (p->infil_on && !(p->dtheta > 0.0)) return SWE_EINVAL;
    if ((size_t)p->nx * (size_t)p->ny > ((size_t)1 << 36)) return SWE_EINVAL;
    return SWE_OK;
}

KParams to_kparams(const swe_params& p) {
    KParams k;
    k.nx = p.nx; k.ny = p.ny;
    k.dx = p.dx; k.dy = p.dy; k.g = p.g; k.cfl = p.cfl; k.dt_max = p.dt_max;
    k.h_eps = p.h_eps;
    k.bcw = p.bc[0]; k.bce = p.bc[1]; k.bcs = p.bc[2]; k.bcn = p.bc[3];
    k.law = p.fric_law; k.coef = p.fric_coef; k.rain = p.rain;
    k.infil = p.infil_on; k.ks = p.ks; k.psi = p.psi; k.dtheta = p.dtheta;
    return k;
}

// Rows per block: enough blocks to fill 256 CUs several times over, at most
// 64 rows (the prologue of each block re-reads two halo rows).
int pick_rows(int nx, int ny) {
    long long strips = (nx + OUT_W - 1) / OUT_W;
    long long ty = (strips * (long long)ny) / 4096;
    if (ty > 64) ty = 64;
    if (ty < 8) ty = 8;
    return (int)ty;
}

dim3 stage_grid(const swe_ctx* c) {
    return dim3((c->prm.nx + OUT_W - 1) / OUT_W, (c->prm.ny + c->ty - 1) / c->ty);
}

int hip_ok(hipError_t e) { return e == hipSuccess ? SWE_OK : SWE_EHIP; }

StageArgs base_args(const swe_ctx* c) {
    StageArgs a;
    std::memset(&a, 0, sizeof a);
    a.p = c->kp;
    a.ty = c->ty;
    a.z = c->buf.z;
    a.fric = c->buf.fric;
    a.vinf = c->buf.vinf;
    a.sc = c->sc;
    a.dtlog = c->dtlog;
    a.dtlog_cap = c->dtlog_cap;
    return a;
}

}  // namespace

extern "C" {

int swe_workspace_bytes(const swe_params* p, size_t* bytes) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!bytes) return SWE_EINVAL;
    size_t n = ncells(p);
    *bytes = 256 + 6 * align256(n * sizeof(double)) +
             align256((size_t)DIAG_BLOCKS * 5 * sizeof(double));
    return SWE_OK;
}

int swe_create(const swe_params* p, const swe_buffers* b, void* workspace,
               size_t workspace_bytes, void* stream, swe_ctx** out) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!b || !out || !workspace || !b->h || !b->qx || !b->qy || !b->z) return SWE_EINVAL;
    if (p->infil_on && !b->vinf) return SWE_EINVAL;
    if (((uintptr_t)workspace & 255) != 0) return SWE_EINVAL;
    size_t need = 0;
    swe_workspace_bytes(p, &need);
    if (workspace_bytes < need) return SWE_ENOMEM;
    swe_ctx* c = new (std::nothrow) swe_ctx;
    if (!c) return SWE_ENOMEM;
    std::memset(c, 0, sizeof *c);
    c->prm = *p;
    c->kp = to_kparams(*p);
    c->buf = *b;
    if (!p->infil_on) c->buf.vinf = nullptr;
    c->stream = (hipStream_t)stream;
    char* w = (char*)workspace;
    size_t n = ncells(p), an = align256(n * sizeof(double));
    c->sc = (DevScalars*)w;
    w += 256;
    c->bh = (double*)w; w += an;
    c->bqx = (double*)w; w += an;
    c->bqy = (double*)w; w += an;
    c->ph = (double*)w; w += an;
    c->pqx = (double*)w; w += an;
    c->pqy = (double*)w; w += an;
    c->diag = (double*)w;
    c->slot = 0;
    c->ty = pick_rows(p->nx, p->ny);
    hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(64), 0, c->stream, c->sc, 0.0);
    rc = hip_ok(hipGetLastError());
    if (rc) { delete c; return rc; }
    *out = c;
    return SWE_OK;
}

int swe_destroy(swe_ctx* c) {
    if (!c) return SWE_OK;
    if (c->prof_ev) {
        for (int k = 0; k < 3 * c->prof_cap; ++k) (void)hipEventDestroy(c->prof_ev[k]);
        delete[] c->prof_ev;
    }
    delete c;
    return SWE_OK;
}

int swe_profile_begin(swe_ctx* c, int32_t max_steps) {
    if (!c || max_steps < 1 || max_steps > (1 << 20) || c->prof_ev) return SWE_EINVAL;
    c->prof_ev = new (std::nothrow) hipEvent_t[3 * (size_t)max_steps];
    if (!c->prof_ev) return SWE_ENOMEM;
    for (int k = 0; k < 3 * max_steps; ++k) {
        if (hipEventCreate(&c->prof_ev[k]) != hipSuccess) {
            for (int j = 0; j < k; ++j) (void)hipEventDestroy(c->prof_ev[j]);
            delete[] c->prof_ev;
            c->prof_ev = nullptr;
            return SWE_EHIP;
        }
    }
    c->prof_cap = max_steps;
    c->prof_n = 0;
    return SWE_OK;
}

int swe_profile_end(swe_ctx* c, double* ms_rate, double* ms_update, int32_t* nsteps) {
    if (!c || !c->prof_ev) return SWE_EINVAL;
    int rc = SWE_OK;
    double a = 0.0, b = 0.0;
    if (hipStreamSynchronize(c->stream) != hipSuccess) rc = SWE_EHIP;
    for (int k = 0; rc == SWE_OK && k < c->prof_n; ++k) {
        float e1 = 0.f, e2 = 0.f;
        if (hipEventElapsedTime(&e1, c->prof_ev[3 * k], c->prof_ev[3 * k + 1]) != hipSuccess ||
            hipEventElapsedTime(&e2, c->prof_ev[3 * k + 1], c->prof_ev[3 * k + 2]) != hipSuccess)
            rc = SWE_EHIP;
        a += e1;
        b += e2;
    }
    if (ms_rate) *ms_rate = a;
    if (ms_update) *ms_update = b;
    if (nsteps) *nsteps = c->prof_n;
    for (int k = 0; k < 3 * c->prof_cap; ++k) (void)hipEventDestroy(c->prof_ev[k]);
    delete[] c->prof_ev;
    c->prof_ev = nullptr;
    c->prof_cap = c->prof_n = 0;
    return rc;
}

int swe_set_time(swe_ctx* c, double t) {
    if (!c || !std::isfinite(t)) return SWE_EINVAL;
    hipLaunchKernelGGL(set_time_kernel, dim3(1), dim3(64), 0, c->stream, c->sc, c->slot, t);
    return hip_ok(hipGetLastError());
}

int swe_set_rain(swe_ctx* c, double rain) {
    if (!c || !(rain >= 0.0) || !std::isfinite(rain)) return SWE_EINVAL;
    c->prm.rain = rain;
    c->kp.rain = rain;
    return SWE_OK;
}

int swe_set_dt_log(swe_ctx* c, double* dev_log, int64_t capacity) {
    if (!c || capacity < 0) return SWE_EINVAL;
    c->dtlog = dev_log;
    c->dtlog_cap = dev_log ? capacity : 0;
    return SWE_OK;
}

int swe_step(swe_ctx* c, int32_t nsteps, double t_end) {
    if (!c || nsteps < 0 || std::isnan(t_end)) return SWE_EINVAL;
    if (nsteps == 0) return SWE_OK;
    dim3 grid = stage_grid(c);
    size_t n = ncells(&c->prm);
    // the state alternates between the caller's buffers (A) and the
    // workspace copy (B); step k reads one and writes the other
    double* Ah = c->buf.h; double* Aqx = c->buf.qx; double* Aqy = c->buf.qy;
    double* Bh = c->bh; double* Bqx = c->bqx; double* Bqy = c->bqy;
    for (int32_t k = 0; k < nsteps; ++k) {
        bool fromA = (k % 2) == 0;
        StageArgs a = base_args(c);
        a.h = fromA ? Ah : Bh;
        a.qx = fromA ? Aqx : Bqx;
        a.qy = fromA ? Aqy : Bqy;
        a.ph = c->ph; a.pqx = c->pqx; a.pqy = c->pqy;
        a.slot = c->slot;
        a.amax_acc = c->sc->amax[c->slot];
        a.amax_clear = c->sc->amax[c->slot ^ 1];
        a.t_end = t_end;
        bool prof = c->prof_ev && c->prof_n < c->prof_cap;
        if (prof) (void)hipEventRecord(c->prof_ev[3 * c->prof_n], c->stream);
        hipLaunchKernelGGL(stage_kernel<1>, grid, dim3(TX), 0, c->stream, a);
        if (prof) (void)hipEventRecord(c->prof_ev[3 * c->prof_n + 1], c->stream);
        a.ho = fromA ? Bh : Ah;
        a.qxo = fromA ? Bqx : Aqx;
        a.qyo = fromA ? Bqy : Aqy;
        hipLaunchKernelGGL(stage_kernel<2>, grid, dim3(TX), 0, c->stream, a);
        if (prof) (void)hipEventRecord(c->prof_ev[3 * c->prof_n++ + 2], c->stream);
        c->slot ^= 1;
    }
    if (nsteps % 2 == 1) {
        hipLaunchKernelGGL(copy3_kernel, dim3(1024), dim3(256), 0, c->stream,
                           (const double*)Bh, (const double*)Bqx, (const double*)Bqy,
                           Ah, Aqx, Aqy, n);
    }
    return hip_ok(hipGetLastError());
}

int swe_get_time(swe_ctx* c, double* t, double* last_dt, int64_t* steps) {
    if (!c) return SWE_EINVAL;
    DevScalars s;
    if (hipMemcpyAsync(&s, c->sc, sizeof s, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return SWE_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SWE_EHIP;
    if (t) *t = s.t[c->slot];
    if (last_dt) *last_dt = s.last_dt;
    if (steps) *steps = s.steps[c->slot];
    return SWE_OK;
}

int swe_get_status(swe_ctx* c, uint32_t* flags) {
    if (!c) return SWE_EINVAL;
    DevScalars s;
    if (hipMemcpyAsync(&s, c->sc, sizeof s, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return SWE_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SWE_EHIP;
    if (flags) *flags = s.status;
    if (s.status & SWE_FLAG_NONFINITE) return SWE_ENONFINITE;
    if (s.status & SWE_FLAG_NEGDEPTH) return SWE_ENEGDEPTH;
    if (s.status & SWE_FLAG_DT) return SWE_EDT;
    return SWE_OK;
}

int swe_get_diagnostics(swe_ctx* c, swe_diag* d) {
    if (!c || !d) return SWE_EINVAL;
    size_t n = ncells(&c->prm);
    hipLaunchKernelGGL(diag_partial_kernel, dim3(DIAG_BLOCKS), dim3(DIAG_T), 0, c->stream,
                       (const double*)c->buf.h, (const double*)c->buf.vinf, c->prm.h_eps, n,
                       c->diag);
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(64), 0, c->stream, c->diag,
                       DIAG_BLOCKS);
    double r[5];
    if (hipMemcpyAsync(r, c->diag, sizeof r, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return SWE_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SWE_EHIP;
    double area = c->prm.dx * c->prm.dy;
    d->mass = r[0] * area;
    d->infiltrated = r[1] * area;
    d->h_min = r[2];
    d->h_max = r[3];
    d->wet_cells = (int64_t)r[4];
    return SWE_OK;
}

int swe_rate(swe_ctx* c, const double* h, const double* qx, const double* qy,
             double* ph, double* pqx, double* pqy, double* amax) {
    if (!c || !h || !qx || !qy || !ph || !pqx || !pqy) return SWE_EINVAL;
    hipLaunchKernelGGL(clear_amax_kernel, dim3(1), dim3(64), 0, c->stream, c->sc, 2);
    StageArgs a = base_args(c);
    a.h = h; a.qx = qx; a.qy = qy;
    a.ph = ph; a.pqx = pqx; a.pqy = pqy;
    // slot 2 of the maxima is reserved for this call and is not a step slot
    a.amax_acc = c->sc->amax[2];
    a.amax_clear = nullptr;
    hipLaunchKernelGGL(stage_kernel<1>, stage_grid(c), dim3(TX), 0, c->stream, a);
    unsigned long long got[2];
    if (hipMemcpyAsync(got, &c->sc->amax[2][0], sizeof got, hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess)
        return SWE_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SWE_EHIP;
    if (amax) {
        std::memcpy(&amax[0], &got[0], 8);
        std::memcpy(&amax[1], &got[1], 8);
    }
    return hip_ok(hipGetLastError());
}

const char* swe_strerror(int code) {
    switch (code) {
        case SWE_OK: return "ok";
        case SWE_EINVAL: return "invalid argument";
        case SWE_EHIP: return "HIP runtime error";
        case SWE_ENEGDEPTH: return "negative water depth produced";
        case SWE_ENONFINITE: return "non-finite value produced";
        case SWE_EDT: return "time step not finite";
        case SWE_ENOMEM: return "workspace too small";
        default: return "unknown error";
    }
}

}  // extern "C"
