// Plain FP64 CPU oracle for the well-balanced 2D Saint-Venant step.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// CPU-baseline leg of the benchmark may load this library.  It shares no code
// with the HIP library: no headers, helpers, tables or constants.
//
// Everything is written from the paper "FullSWOF_Paral" (Cordier, Coullon,
// Delestre, Laguerre, Le, Pierre, Sadaka; arXiv:1307.4839) as plain loops in
// the order the paper states the method:
//   * model (SW2D), Section 2.1: mass + two momentum laws, g = 9.81, rain R,
//     infiltration I, Manning and Darcy-Weisbach friction laws;
//   * Section 3.1 (eq. SW1Dscheme): finite-volume convective step with the
//     hydrostatic reconstruction, the interface corrections S and the
//     centred source Fc;
//   * Section 3.2: semi-implicit friction and Heun's two-stage RK2;
//   * Section 3.3: HLL flux with c1/c2 wave-speed bounds, CFL (eq. cfl) on
//     the reconstructed states at second order;
//   * Section 3.4: MUSCL with minmod on h, h+z and u, with the modified
//     velocity reconstruction that conserves discharge;
//   * Section 3.5: modified Green-Ampt infiltration;
//   * Section 6.2, Algorithm 1: order of operations inside a stage
//     (boundary conditions, reconstruction, hydrostatic reconstruction, flux,
//     scheme, friction), then Heun's combination;
//   * Section 2.2: boundary values given by ghost cells; Section 6.1: two
//     ghost layers at second order.
//
// Readings where the paper is silent (2D extension, dry threshold, friction
// in 2D, Manning form, rain/infiltration placement, Green-Ampt constants,
// ghost definitions, time-step bound in 2D) are the documented readings of
// the project; each is marked "reading:" where it is used.
//
// The arithmetic is templated on the scalar type T so that the same code can
// run in double (the oracle) and with a forward-mode dual number (the
// tangent used to pin the adjoint).  Nothing here is blocked, fused or
// reordered beyond what the formulas say; rows are distributed over OpenMP
// threads, which does not change any result because every cell update is
// independent once the time step is known and a maximum is exact.

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Scalar types
// ---------------------------------------------------------------------------

// Forward-mode dual number: value v and one directional derivative d.
struct Dual {
    double v, d;
    Dual() : v(0), d(0) {}
    Dual(double x) : v(x), d(0) {}
    Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
    double q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
inline Dual dsqrt(Dual a) {
    double s = std::sqrt(a.v);
    return Dual(s, s > 0 ? a.d / (2.0 * s) : 0.0);
}
inline Dual dcbrt(Dual a) {
    double c = std::cbrt(a.v);
    return Dual(c, c != 0 ? a.d / (3.0 * c * c) : 0.0);
}
inline Dual dfabs(Dual a) { return a.v < 0 ? -a : a; }
inline double val(Dual a) { return a.v; }
inline double der(Dual a) { return a.d; }

inline double dsqrt(double a) { return std::sqrt(a); }
inline double dcbrt(double a) { return std::cbrt(a); }
inline double dfabs(double a) { return std::fabs(a); }
inline double val(double a) { return a; }
inline double der(double) { return 0.0; }

// max/min that return one of their arguments; on a tie the first one.
template <class T> inline T vmax(T a, T b) { return (a < b) ? b : a; }
template <class T> inline T vmin(T a, T b) { return (b < a) ? b : a; }

// ---------------------------------------------------------------------------
// Parameters (own definition; mirrors nothing)
// ---------------------------------------------------------------------------

enum { BC_WALL = 0, BC_OUTFLOW = 1, BC_IMPOSED_H = 2, BC_IMPOSED_Q = 3, BC_IMPOSED_HQ = 4 };
enum { LAW_NONE = 0, LAW_MANNING = 1, LAW_DARCY = 2 };

}  // namespace

extern "C" {
struct orc_params {
    int32_t nx, ny;
    double dx, dy;
    double g;
    double cfl;
    double dt_max;
    double h_eps;
    int32_t bc[4];  // west, east, south, north
    int32_t fric_law;
    double fric_coef;
    double rain;
    int32_t infil_on;
    double ks, psi, dtheta;
    // R(t, x, y) = r(t) w(x, y) (Section 2.1 lets rain vary in time and
    // space).  r(t) is the piecewise-constant hyetograph: r_k from t_k up to
    // t_{k+1}, 0 before t_0; with rain_n = 0 it is the constant `rain`.
    int32_t rain_n;
    const double* rain_t;
    const double* rain_r;
    const double* rain_w;    // per-cell weight w, or NULL for 1
    // per-cell Green-Ampt parameters (Section 3.5), or NULL for the scalars
    const double* ks_f;
    const double* psi_f;
    const double* dtheta_f;
    // 1: first order (Section 3.3: piecewise-constant reconstruction, one
    // explicit Euler stage per step); 0 or 2: the second-order scheme
    int32_t order;
    // numerical flux (Section 3.3 allows any consistent one): 0 HLL, 1 Rusanov,
    // 2 kinetic, 3 VFRoe-ncv
    int32_t flux;
    // imposed boundaries (bc 2: depth h_b, 3: inflow discharge q_b per unit
    // width, 4: both), per side west, east, south, north
    double bc_h[4];
    double bc_q[4];
    // smallest acceptable time step (0: none): a dt of eq. (cfl) below it,
    // other than the last step clipped to the end time, is a collapse of the
    // time step and stops the run before that step
    double dt_min;
    // second-order reconstruction (Section 4.1 lists MUSCL, ENO and modified
    // ENO): 0 MUSCL with minmod, 1 ENO, 2 modified ENO; ignored at order 1
    int32_t recon;
};
}

namespace {

// ---------------------------------------------------------------------------
// Section 3.4: minmod limiter and MUSCL reconstruction of one cell
// ---------------------------------------------------------------------------

// minmod(x, y) = min if both >= 0, max if both <= 0, else 0 (Section 3.4).
template <class T> inline T minmod(T a, T b) {
    if (a >= T(0.0) && b >= T(0.0)) return vmin(a, b);
    if (a <= T(0.0) && b <= T(0.0)) return vmax(a, b);
    return T(0.0);
}

// Reconstructed values of one cell at its two faces along one direction.
// "m" is the face at i-1/2 (the value s_{i-1/2+}), "p" the face at i+1/2
// (the value s_{i+1/2-}).  un is the velocity normal to the faces, ut the
// tangential one.
template <class T> struct Recon {
    T h_m, h_p, z_m, z_p, un_m, un_p, ut_m, ut_p;
};

// Primitive variables of one cell (Section 3.1: MUSCL acts on u, h, h+z).
template <class T> struct Prim {
    T h, un, ut, eta;
};

// Section 3.4.  The limiter is applied to the undivided differences
// (reading: s -/+ (dx/2) Ds with Ds = minmod of divided differences equals
// s -/+ minmod(undivided)/2 in exact arithmetic).  z is deduced from the
// reconstructions of h and h+z.  The velocity reconstruction is the modified
// one that conserves discharge; for a cell at or below the dry threshold the
// velocity is not reconstructed (reading: the formula divides by h_i).
template <class T>
inline Recon<T> muscl(const Prim<T>& a, const Prim<T>& c, const Prim<T>& b,
                      double h_eps) {
    Recon<T> r;
    T dh = minmod(c.h - a.h, b.h - c.h);
    r.h_m = c.h - T(0.5) * dh;
    r.h_p = c.h + T(0.5) * dh;
    T de = minmod(c.eta - a.eta, b.eta - c.eta);
    T eta_m = c.eta - T(0.5) * de;
    T eta_p = c.eta + T(0.5) * de;
    r.z_m = eta_m - r.h_m;
    r.z_p = eta_p - r.h_p;
    T dun = minmod(c.un - a.un, b.un - c.un);
    T dut = minmod(c.ut - a.ut, b.ut - c.ut);
    if (c.h > T(h_eps)) {
        // u_{i-1/2+} = u_i - (h_{i+1/2-}/h_i) (dx/2) Du_i and
        // u_{i+1/2-} = u_i + (h_{i-1/2+}/h_i) (dx/2) Du_i.
        r.un_m = c.un - (r.h_p / c.h) * (T(0.5) * dun);
        r.un_p = c.un + (r.h_m / c.h) * (T(0.5) * dun);
        r.ut_m = c.ut - (r.h_p / c.h) * (T(0.5) * dut);
        r.ut_p = c.ut + (r.h_m / c.h) * (T(0.5) * dut);
    } else {
        r.un_m = r.un_p = c.un;
        r.ut_m = r.ut_p = c.ut;
    }
    return r;
}

// ENO reconstruction at second order (Section 4.1 names ENO and modified ENO
// beside MUSCL without defining them; reading).  Every second-order
// reconstruction of the paper works on the cells i-1, i, i+1 (two ghost
// layers at order two, Section 6.1), so ENO is Harten's at second order:
// of the two two-cell stencils the smoother one, i.e. the one-sided
// undivided difference of smaller magnitude (the left one on ties), as the
// slope of h, h+z and the velocities.  Unlike minmod it keeps a slope at an
// extremum, and the face depths h -/+ D/2 can then be negative.  A cell at
// or below the dry threshold keeps its values at both faces (its slopes
// would put water on the faces of a dry cell between wet ones; the same
// threshold stops the velocity reconstruction of MUSCL).  Modified ENO: the
// same with the depth's slope limited to |D| <= 2 h_i, so that both face
// depths stay in [0, 2 h_i], as the positivity of the hydrostatic
// reconstruction (Section 3.1) needs.  z and the velocities follow as for
// MUSCL (modified velocity conserving the discharge).
template <class T> inline T eno_slope(T a, T b) { return dfabs(a) <= dfabs(b) ? a : b; }

template <class T>
inline Recon<T> eno(const Prim<T>& a, const Prim<T>& c, const Prim<T>& b, double h_eps,
                    bool modified) {
    Recon<T> r;
    if (!(c.h > T(h_eps))) {
        r.h_m = r.h_p = c.h;
        r.z_m = r.z_p = c.eta - c.h;
        r.un_m = r.un_p = c.un;
        r.ut_m = r.ut_p = c.ut;
        return r;
    }
    T dh = eno_slope(c.h - a.h, b.h - c.h);
    if (modified) {
        T cap = T(2.0) * c.h;
        if (dh > cap) dh = cap;
        else if (dh < -cap) dh = -cap;
    }
    r.h_m = c.h - T(0.5) * dh;
    r.h_p = c.h + T(0.5) * dh;
    T de = eno_slope(c.eta - a.eta, b.eta - c.eta);
    T eta_m = c.eta - T(0.5) * de;
    T eta_p = c.eta + T(0.5) * de;
    r.z_m = eta_m - r.h_m;
    r.z_p = eta_p - r.h_p;
    T dun = eno_slope(c.un - a.un, b.un - c.un);
    T dut = eno_slope(c.ut - a.ut, b.ut - c.ut);
    r.un_m = c.un - (r.h_p / c.h) * (T(0.5) * dun);
    r.un_p = c.un + (r.h_m / c.h) * (T(0.5) * dun);
    r.ut_m = c.ut - (r.h_p / c.h) * (T(0.5) * dut);
    r.ut_p = c.ut + (r.h_m / c.h) * (T(0.5) * dut);
    return r;
}

// First order (Section 3.3 gives n_CFL = 1 for it): no reconstruction, the
// face values are the cell's.  Written as the reconstruction above with
// zero slopes, so z at the faces is still deduced from h and h+z.
template <class T>
inline Recon<T> piecewise_constant(const Prim<T>& c) {
    Recon<T> r;
    r.h_m = r.h_p = c.h;
    r.z_m = r.z_p = c.eta - c.h;
    r.un_m = r.un_p = c.un;
    r.ut_m = r.ut_p = c.ut;
    return r;
}

// The face values of one cell for the parameters' order and reconstruction.
template <class T>
inline Recon<T> reconstruct(const orc_params& p, const Prim<T>& a, const Prim<T>& c,
                            const Prim<T>& b) {
    if (p.order == 1) return piecewise_constant(c);
    if (p.recon == 1 || p.recon == 2) return eno(a, c, b, p.h_eps, p.recon == 2);
    return muscl(a, c, b, p.h_eps);
}

// ---------------------------------------------------------------------------
// Section 3.3: HLL flux of the homogeneous system along the face normal
// ---------------------------------------------------------------------------

// Physical flux F(U) = (h un, h un^2 + g h^2/2, h un ut) along the normal.
// Returns (mass, normal momentum, tangential momentum).
template <class T>
inline void hll(double g, T hL, T unL, T utL, T hR, T unR, T utR, T F[3]) {
    T cL = dsqrt(T(g) * hL);
    T cR = dsqrt(T(g) * hR);
    // c1 = inf of the eigenvalues u -/+ sqrt(gh) over U_L, U_R; c2 = sup.
    T c1 = vmin(unL - cL, unR - cR);
    T c2 = vmax(unL + cL, unR + cR);
    T qL = hL * unL;
    T qR = hR * unR;
    T FL[3] = {qL, qL * unL + T(0.5 * g) * hL * hL, qL * utL};
    T FR[3] = {qR, qR * unR + T(0.5 * g) * hR * hR, qR * utR};
    if (T(0.0) <= c1) {
        for (int k = 0; k < 3; ++k) F[k] = FL[k];
    } else if (c2 <= T(0.0)) {
        for (int k = 0; k < 3; ++k) F[k] = FR[k];
    } else {
        T UL[3] = {hL, qL, hL * utL};
        T UR[3] = {hR, qR, hR * utR};
        for (int k = 0; k < 3; ++k)
            F[k] = (c2 * FL[k] - c1 * FR[k]) / (c2 - c1) +
                   c1 * c2 / (c2 - c1) * (UR[k] - UL[k]);
    }
}

// Rusanov (local Lax-Friedrichs) flux, one of the consistent fluxes
// Section 3.3 lists: the centred average of the physical fluxes minus a
// diffusion with the largest local wave speed,
//   F = (F(U_L) + F(U_R))/2 - c/2 (U_R - U_L),
//   c = max(|u_L| + sqrt(g h_L), |u_R| + sqrt(g h_R)).
template <class T>
inline void rusanov(double g, T hL, T unL, T utL, T hR, T unR, T utR, T F[3]) {
    T cL = dsqrt(T(g) * hL);
    T cR = dsqrt(T(g) * hR);
    T c = vmax(dfabs(unL) + cL, dfabs(unR) + cR);
    T qL = hL * unL;
    T qR = hR * unR;
    T FL[3] = {qL, qL * unL + T(0.5 * g) * hL * hL, qL * utL};
    T FR[3] = {qR, qR * unR + T(0.5 * g) * hR * hR, qR * utR};
    T UL[3] = {hL, qL, hL * utL};
    T UR[3] = {hR, qR, hR * utR};
    for (int k = 0; k < 3; ++k)
        F[k] = T(0.5) * (FL[k] + FR[k]) - T(0.5) * c * (UR[k] - UL[k]);
}

// Kinetic flux (Perthame and Simeoni, 2001; Audusse, Bristeau and Perthame,
// 2000), another flux Section 3.3 lists.  A state (h, u) is the mean of
// particles whose velocities xi spread uniformly over [u - s, u + s],
// s = sqrt(3 g h / 2), with density h / (2 s): their moments are h, h u and
// h u^2 + g h^2 / 2.  Particles with xi > 0 cross the face from the left
// state and those with xi < 0 from the right one:
//   F_h = int_{xi > 0} xi M_L + int_{xi < 0} xi M_R,
//   F_q = int_{xi > 0} xi^2 M_L + int_{xi < 0} xi^2 M_R,
// and the tangential momentum rides with the mass each side sends.  Over
// [a, b]: int xi = (b^2 - a^2) / 2 and int xi^2 = (b^3 - a^3) / 3.  A dry
// side (h = 0) sends nothing.
template <class T>
inline void kinetic_half(double g, T h, T un, bool left, T& m0, T& m1) {
    if (!(h > T(0.0))) {
        m0 = T(0.0);
        m1 = T(0.0);
        return;
    }
    T s = dsqrt(T(1.5 * g) * h);
    T a = un - s;
    T b = un + s;
    if (left) {
        a = vmax(a, T(0.0));
        b = vmax(b, T(0.0));
    } else {
        a = vmin(a, T(0.0));
        b = vmin(b, T(0.0));
    }
    m0 = (h * (b * b - a * a)) / (T(4.0) * s);
    m1 = (h * (b * b * b - a * a * a)) / (T(6.0) * s);
}

template <class T>
inline void kinetic(double g, T hL, T unL, T utL, T hR, T unR, T utR, T F[3]) {
    T m0L, m1L, m0R, m1R;
    kinetic_half(g, hL, unL, true, m0L, m1L);
    kinetic_half(g, hR, unR, false, m0R, m1R);
    F[0] = m0L + m0R;
    F[1] = m1L + m1R;
    F[2] = m0L * utL + m0R * utR;
}

// VFRoe-ncv flux (Buffard, Gallouet and Herard, 2000; Gallouet, Herard and
// Seguin, 2003), the fourth flux Section 4.1 lists: the interface value of
// the Riemann problem of the system written in the non-conservative
// variables W = (2c, u), c = sqrt(g h),
//   (2c)_t + u (2c)_x + c u_x = 0,   u_t + c (2c)_x + u u_x = 0,
// linearized about the mean state (c^, u^) = ((cL + cR)/2, (uL + uR)/2).
// Its eigenvalues are u^ -/+ c^ and 2c - u, 2c + u are carried along them.
// At x/t = 0: W_L if u^ - c^ >= 0, W_R if u^ + c^ <= 0, else the state with
// 2c* + u* = 2cL + uL and 2c* - u* = 2cR - uR:
//   c* = c^ + (uL - uR)/4,   u* = u^ + (cL - cR).
// The face flux is the physical flux of that state, with h* = max(c*, 0)^2 / g
// (the depth of U_L or U_R itself in the outer branches), and the
// tangential velocity upwinded on u* (left side when u* >= 0).  Readings for
// dry sides, where W holds a velocity that carries no water: a dry side
// takes the other side's velocity, and two dry sides pass nothing.
template <class T>
inline void vfroe(double g, T hL, T unL, T utL, T hR, T unR, T utR, T F[3]) {
    const bool wetL = hL > T(0.0), wetR = hR > T(0.0);
    if (!wetL && !wetR) {
        F[0] = F[1] = F[2] = T(0.0);
        return;
    }
    if (!wetL) unL = unR;
    if (!wetR) unR = unL;
    T cL = dsqrt(T(g) * hL);
    T cR = dsqrt(T(g) * hR);
    T uh = T(0.5) * (unL + unR);
    T ch = T(0.5) * (cL + cR);
    T h, u;
    if (uh - ch >= T(0.0)) {
        h = hL;
        u = unL;
    } else if (uh + ch <= T(0.0)) {
        h = hR;
        u = unR;
    } else {
        T cs = vmax(ch + T(0.25) * (unL - unR), T(0.0));
        h = (cs * cs) / T(g);
        u = uh + (cL - cR);
    }
    T q = h * u;
    F[0] = q;
    F[1] = q * u + T(0.5 * g) * h * h;
    F[2] = q * (u >= T(0.0) ? utL : utR);
}

// One face between a left cell (its "p" values) and a right cell (its "m"
// values): hydrostatic reconstruction (Section 3.1), HLL (Rusanov, kinetic,
// VFRoe-ncv) flux and the two
// normal-momentum corrections S_{i+1/2L} (for the left cell) and
// S_{i+1/2R} (for the right cell).  Also returns the face's wave-speed bound
// max(|u-| + sqrt(g h-), |u+| + sqrt(g h+)) on the MUSCL states, i.e. before
// the hydrostatic reconstruction (eq. cfl and the remark after it); with
// the kinetic flux the bound is the particles' largest speed,
// max(|u-| + sqrt(3 g h- / 2), |u+| + sqrt(3 g h+ / 2)).
template <class T> struct Face {
    T F[3];
    T sL, sR;
    double speed;
};

template <class T>
inline Face<T> face(double g, T hm, T zm, T unm, T utm, T hp, T zp, T unp,
                    T utp, int flux = 0) {
    Face<T> f;
    T zs = vmax(zm, zp);
    T hL = vmax(hm + zm - zs, T(0.0));
    T hR = vmax(hp + zp - zs, T(0.0));
    // U_L = (h_L, h_L u-), U_R = (h_R, h_R u+); in 2D the tangential
    // velocity is carried the same way (reading).
    if (flux == 1)
        rusanov(g, hL, unm, utm, hR, unp, utp, f.F);
    else if (flux == 2)
        kinetic(g, hL, unm, utm, hR, unp, utp, f.F);
    else if (flux == 3)
        vfroe(g, hL, unm, utm, hR, unp, utp, f.F);
    else
        hll(g, hL, unm, utm, hR, unp, utp, f.F);
    f.sL = T(0.5 * g) * (hm * hm - hL * hL);
    f.sR = T(0.5 * g) * (hp * hp - hR * hR);
    const double gs = flux == 2 ? 1.5 * g : g;
    double sm = std::fabs(val(unm)) + std::sqrt(gs * val(hm));
    double sp = std::fabs(val(unp)) + std::sqrt(gs * val(hp));
    f.speed = sm < sp ? sp : sm;
    return f;
}

// ---------------------------------------------------------------------------
// Grid with two ghost layers (Section 2.2 and Section 6.1)
// ---------------------------------------------------------------------------

const int G = 2;  // ghost width at second order

struct Grid {
    int nx, ny, px, py;
    Grid(int nx_, int ny_) : nx(nx_), ny(ny_), px(nx_ + 2 * G), py(ny_ + 2 * G) {}
    // index of cell (i, j), i in [-G, nx+G), j in [-G, ny+G)
    size_t at(int i, int j) const { return (size_t)(j + G) * px + (i + G); }
    size_t size() const { return (size_t)px * py; }
};

// Imposed boundary (Section 2.2): the ghost state comes from the Riemann
// invariants.  With w the outward normal velocity of the boundary cell and
// c = sqrt(g h), the invariant w + 2c is carried out of the domain by the
// characteristic w + c, so the ghost keeps it.  In fluvial flow one
// variable is imposed: the depth h_b (w of the ghost from the invariant) or
// the inflow discharge q_b (the depth from the invariant); with both
// imposed (supercritical inflow) the ghost is (h_b, q_b); a boundary cell in
// supercritical outflow (w > c) is free (the ghost copies it).  The ghost
// keeps the boundary cell's tangential velocity.  Inputs and outputs: depth,
// outward normal discharge, tangential discharge.
template <class T>
inline void imposed_ghost(const orc_params& p, int side, T hb, T qo, T qt, T& hg, T& qog,
                          T& qtg) {
    const double g = p.g;
    const bool wet = hb > T(p.h_eps);
    T w = wet ? qo / hb : T(0.0);
    T vt = wet ? qt / hb : T(0.0);
    T c = dsqrt(T(g) * hb);
    if (w > c) {  // supercritical outflow: free
        hg = hb;
        qog = qo;
        qtg = qt;
        return;
    }
    const int type = p.bc[side];
    if (type == BC_IMPOSED_HQ) {
        hg = T(p.bc_h[side]);
        qog = -T(p.bc_q[side]);
    } else if (type == BC_IMPOSED_H) {
        hg = T(p.bc_h[side]);
        T wg = (w + T(2.0) * c) - T(2.0) * dsqrt(T(g) * hg);
        qog = hg * wg;
    } else {
        // depth of the ghost: 2 sqrt(g h) - q_b / h = w + 2c, increasing in
        // h for q_b >= 0; bisection (bracket doubled from 1 m, then halved
        // 100 times), which only compares, adds, divides and takes roots
        const double qb = p.bc_q[side];
        const double R = val(w + T(2.0) * c);
        auto F = [&](double x) { return 2.0 * std::sqrt(g * x) - qb / x; };
        double hi = 1.0;
        for (int k = 0; k < 200 && F(hi) < R; ++k) hi = 2.0 * hi;
        double lo = 0.0;
        for (int k = 0; k < 100; ++k) {
            double mid = 0.5 * (lo + hi);
            if (F(mid) < R) lo = mid; else hi = mid;
        }
        hg = T(hi);
        qog = -T(qb);
    }
    qtg = hg * vt;
}

// Ghost cells (reading of Section 2.2).  Wall: ghost k mirrors interior
// cell k (h, z and tangential discharge), normal discharge negated.  Free
// outflow: ghosts copy the boundary cell (zero gradient).  Imposed: both
// ghosts take imposed_ghost() of the boundary cell, z copied.  The x-sweep
// reads only x-ghosts and the y-sweep only y-ghosts, so corners are never
// used.
template <class T>
void fill_ghosts(const orc_params& p, const Grid& gr, std::vector<T>& h,
                 std::vector<T>& qx, std::vector<T>& qy, std::vector<T>& z) {
    const int nx = gr.nx, ny = gr.ny;
    auto imposed = [&](int side, size_t dst, size_t src) {
        // outward normal: -x, +x, -y, +y for west, east, south, north
        const bool xn = side < 2;
        const double sg = (side == 0 || side == 2) ? -1.0 : 1.0;
        T qn = xn ? qx[src] : qy[src];
        T qt = xn ? qy[src] : qx[src];
        T hg, qog, qtg;
        imposed_ghost(p, side, h[src], T(sg) * qn, qt, hg, qog, qtg);
        h[dst] = hg;
        z[dst] = z[src];
        if (xn) { qx[dst] = T(sg) * qog; qy[dst] = qtg; }
        else { qy[dst] = T(sg) * qog; qx[dst] = qtg; }
    };
    for (int j = 0; j < ny; ++j) {
        for (int k = 0; k < G; ++k) {
            // west: ghost -1-k
            {
                size_t dst = gr.at(-1 - k, j);
                size_t src = p.bc[0] == BC_WALL ? gr.at(k, j) : gr.at(0, j);
                if (p.bc[0] >= BC_IMPOSED_H) {
                    imposed(0, dst, src);
                } else {
                    h[dst] = h[src]; z[dst] = z[src]; qy[dst] = qy[src];
                    qx[dst] = p.bc[0] == BC_WALL ? -qx[src] : qx[src];
                }
            }
            // east: ghost nx+k
            {
                size_t dst = gr.at(nx + k, j);
                size_t src = p.bc[1] == BC_WALL ? gr.at(nx - 1 - k, j) : gr.at(nx - 1, j);
                if (p.bc[1] >= BC_IMPOSED_H) {
                    imposed(1, dst, src);
                } else {
                    h[dst] = h[src]; z[dst] = z[src]; qy[dst] = qy[src];
                    qx[dst] = p.bc[1] == BC_WALL ? -qx[src] : qx[src];
                }
            }
        }
    }
    for (int i = 0; i < nx; ++i) {
        for (int k = 0; k < G; ++k) {
            // south: ghost -1-k
            {
                size_t dst = gr.at(i, -1 - k);
                size_t src = p.bc[2] == BC_WALL ? gr.at(i, k) : gr.at(i, 0);
                if (p.bc[2] >= BC_IMPOSED_H) {
                    imposed(2, dst, src);
                } else {
                    h[dst] = h[src]; z[dst] = z[src]; qx[dst] = qx[src];
                    qy[dst] = p.bc[2] == BC_WALL ? -qy[src] : qy[src];
                }
            }
            // north: ghost ny+k
            {
                size_t dst = gr.at(i, ny + k);
                size_t src = p.bc[3] == BC_WALL ? gr.at(i, ny - 1 - k) : gr.at(i, ny - 1);
                if (p.bc[3] >= BC_IMPOSED_H) {
                    imposed(3, dst, src);
                } else {
                    h[dst] = h[src]; z[dst] = z[src]; qx[dst] = qx[src];
                    qy[dst] = p.bc[3] == BC_WALL ? -qy[src] : qy[src];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Section 3.1 in 2D: the rate Phi(U) of one convective stage
// ---------------------------------------------------------------------------
//
// Reading of the 2D extension by the method of lines: the x-faces and the
// y-faces contribute in one unsplit update,
//   Phi = -( X / dx + Y / dy ),
// where X = F_{i+1/2L} - F_{i-1/2R} - Fc_i with the x-normal momentum
// carrying S and Fc, and Y is the same along y.  A stage is
// U* = U + dt Phi(U) (Section 3.2, Heun).

template <class T>
void rate(const orc_params& p, const T* h_in, const T* qx_in, const T* qy_in,
          const double* z_in, T* ph, T* pqx, T* pqy, double amax[2]) {
    const int nx = p.nx, ny = p.ny;
    const double g = p.g, h_eps = p.h_eps;
    Grid gr(nx, ny);
    std::vector<T> h(gr.size()), qx(gr.size()), qy(gr.size()), z(gr.size());
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t s = (size_t)j * nx + i, d = gr.at(i, j);
            h[d] = h_in[s]; qx[d] = qx_in[s]; qy[d] = qy_in[s]; z[d] = T(z_in[s]);
        }
    // O1: boundary conditions
    fill_ghosts(p, gr, h, qx, qy, z);

    // O2: primitive variables; velocity is 0 at or below the dry threshold
    // (reading).
    std::vector<T> u(gr.size()), v(gr.size()), eta(gr.size());
    for (size_t k = 0; k < gr.size(); ++k) {
        if (h[k] > T(h_eps)) {
            u[k] = qx[k] / h[k];
            v[k] = qy[k] / h[k];
        } else {
            u[k] = T(0.0);
            v[k] = T(0.0);
        }
        eta[k] = h[k] + z[k];
    }

    std::vector<T> X0((size_t)nx * ny), X1((size_t)nx * ny), X2((size_t)nx * ny);
    std::vector<T> Y0((size_t)nx * ny), Y1((size_t)nx * ny), Y2((size_t)nx * ny);
    double ax = 0.0, ay = 0.0;

    // x-sweep: each row j is a 1D problem with normal velocity u.
#pragma omp parallel for schedule(static) reduction(max : ax)
    for (int j = 0; j < ny; ++j) {
        // reconstruct cells -1 .. nx (indices shifted by +1)
        std::vector<Recon<T>> rc(nx + 2);
        for (int i = -1; i <= nx; ++i) {
            size_t a = gr.at(i - 1, j), c = gr.at(i, j), b = gr.at(i + 1, j);
            Prim<T> pa{h[a], u[a], v[a], eta[a]};
            Prim<T> pc{h[c], u[c], v[c], eta[c]};
            Prim<T> pb{h[b], u[b], v[b], eta[b]};
            rc[i + 1] = reconstruct(p, pa, pc, pb);
        }
        // faces i+1/2 for i = -1 .. nx-1
        std::vector<Face<T>> fc(nx + 1);
        for (int i = -1; i < nx; ++i) {
            const Recon<T>& L = rc[i + 1];
            const Recon<T>& R = rc[i + 2];
            fc[i + 1] = face(g, L.h_p, L.z_p, L.un_p, L.ut_p, R.h_m, R.z_m,
                             R.un_m, R.ut_m, p.flux);
            if (fc[i + 1].speed > ax) ax = fc[i + 1].speed;
        }
        for (int i = 0; i < nx; ++i) {
            const Face<T>& fm = fc[i];      // face i-1/2
            const Face<T>& fp = fc[i + 1];  // face i+1/2
            const Recon<T>& r = rc[i + 1];
            // Fc_i = -g (h_{i-1/2+} + h_{i+1/2-})/2 (z_{i+1/2-} - z_{i-1/2+})
            T fcen = T(-g) * (T(0.5) * (r.h_m + r.h_p)) * (r.z_p - r.z_m);
            size_t s = (size_t)j * nx + i;
            X0[s] = fp.F[0] - fm.F[0];
            X1[s] = (fp.F[1] + fp.sL) - (fm.F[1] + fm.sR) - fcen;
            X2[s] = fp.F[2] - fm.F[2];
        }
    }

    // y-sweep: each column i is a 1D problem with normal velocity v.
#pragma omp parallel for schedule(static) reduction(max : ay)
    for (int i = 0; i < nx; ++i) {
        std::vector<Recon<T>> rc(ny + 2);
        for (int j = -1; j <= ny; ++j) {
            size_t a = gr.at(i, j - 1), c = gr.at(i, j), b = gr.at(i, j + 1);
            Prim<T> pa{h[a], v[a], u[a], eta[a]};
            Prim<T> pc{h[c], v[c], u[c], eta[c]};
            Prim<T> pb{h[b], v[b], u[b], eta[b]};
            rc[j + 1] = reconstruct(p, pa, pc, pb);
        }
        std::vector<Face<T>> fc(ny + 1);
        for (int j = -1; j < ny; ++j) {
            const Recon<T>& L = rc[j + 1];
            const Recon<T>& R = rc[j + 2];
            fc[j + 1] = face(g, L.h_p, L.z_p, L.un_p, L.ut_p, R.h_m, R.z_m,
                             R.un_m, R.ut_m, p.flux);
            if (fc[j + 1].speed > ay) ay = fc[j + 1].speed;
        }
        for (int j = 0; j < ny; ++j) {
            const Face<T>& fm = fc[j];
            const Face<T>& fp = fc[j + 1];
            const Recon<T>& r = rc[j + 1];
            T fcen = T(-g) * (T(0.5) * (r.h_m + r.h_p)) * (r.z_p - r.z_m);
            size_t s = (size_t)j * nx + i;
            Y0[s] = fp.F[0] - fm.F[0];
            Y1[s] = (fp.F[1] + fp.sL) - (fm.F[1] + fm.sR) - fcen;  // normal = qy
            Y2[s] = fp.F[2] - fm.F[2];                             // tangential = qx
        }
    }

    for (size_t s = 0; s < (size_t)nx * ny; ++s) {
        ph[s] = -(X0[s] / T(p.dx) + Y0[s] / T(p.dy));
        pqx[s] = -(X1[s] / T(p.dx) + Y2[s] / T(p.dy));
        pqy[s] = -(X2[s] / T(p.dx) + Y1[s] / T(p.dy));
    }
    if (amax) {
        amax[0] = ax;
        amax[1] = ay;
    }
}

// ---------------------------------------------------------------------------
// Section 3.2: semi-implicit friction of one stage
// ---------------------------------------------------------------------------
//
// (h0, q0) is the stage input ("n"), (h1, q1) the convective output ("*").
// Darcy-Weisbach as printed: q <- q* / (1 + dt (f/8) |q^n| / (h^n h*)).
// Manning by the same split of S_f = n^2 |u| u / h^{4/3} (reading):
//   q <- q* / (1 + dt g n^2 |q^n| / (h^n (h*)^{4/3})).
// In 2D |q| = sqrt(qx^2 + qy^2) and both components share the factor
// (reading).  A cell whose stage output is at or below the dry threshold
// carries no discharge; a cell that was dry at the stage input gets no
// friction in that stage (readings).
template <class T> inline T coef_at(const orc_params& p, const T* fric, size_t s) {
    return fric ? fric[s] : T(p.fric_coef);
}

template <class T>
inline void friction_t(const orc_params& p, T coef, T h0, T qx0, T qy0, T h1,
                       T& qx1, T& qy1, double dt) {
    if (h1 <= T(p.h_eps)) {
        qx1 = T(0.0);
        qy1 = T(0.0);
        return;
    }
    if (p.fric_law == LAW_NONE || !(h0 > T(p.h_eps))) return;
    T qn = dsqrt(qx0 * qx0 + qy0 * qy0);
    T den;
    if (p.fric_law == LAW_DARCY) {
        den = T(1.0) + T(dt) * (coef / T(8.0)) * qn / (h0 * h1);
    } else {
        den = T(1.0) + T(dt) * T(p.g) * coef * coef * qn / (h0 * (h1 * dcbrt(h1)));
    }
    qx1 = qx1 / den;
    qy1 = qy1 / den;
}

// One stage: U_out = friction(U + dt Phi(U)).  Returns amax of the input.
template <class T>
void stage(const orc_params& p, const T* fric, double dt, const T* h,
           const T* qx, const T* qy, const double* z, T* ho, T* qxo, T* qyo,
           double amax[2]) {
    size_t n = (size_t)p.nx * p.ny;
    std::vector<T> ph(n), pqx(n), pqy(n);
    rate(p, h, qx, qy, z, ph.data(), pqx.data(), pqy.data(), amax);
    for (size_t s = 0; s < n; ++s) {
        T h1 = h[s] + T(dt) * ph[s];
        T qx1 = qx[s] + T(dt) * pqx[s];
        T qy1 = qy[s] + T(dt) * pqy[s];
        friction_t(p, coef_at(p, fric, s), h[s], qx[s], qy[s], h1, qx1, qy1, dt);
        ho[s] = h1;
        qxo[s] = qx1;
        qyo[s] = qy1;
    }
}

// Time step from the wave-speed bounds (eq. cfl in 2D, reading):
//   dt = min(dt_max, cfl / (Ax/dx + Ay/dy), t_end - t);
// with no wave (all dry) the bound is dt_max alone.
double time_step(const orc_params& p, const double amax[2], double t, double t_end) {
    double r = amax[0] / p.dx + amax[1] / p.dy;
    double dt = p.dt_max;
    if (r > 0.0) {
        double c = p.cfl / r;
        if (c < dt) dt = c;
    }
    double rest = t_end - t;
    if (rest < dt) dt = rest;
    return dt;
}

// Rain intensity r(t) of the hyetograph at the start time t of a step
// (rain is explicit, Section 3.1): the last breakpoint at or before t.
inline double rain_rate(const orc_params& p, double t) {
    if (p.rain_n <= 0) return p.rain;
    double r = 0.0;
    for (int32_t k = 0; k < p.rain_n; ++k)
        if (p.rain_t[k] <= t) r = p.rain_r[k];
    return r;
}

// Once per step after Heun's combination (reading): explicit rain, then the
// modified Green-Ampt model of Section 3.5 with A = 1 and the capillary term
// read as (psi + h_over)/Z_f with psi >= 0 the suction head.  The water that
// infiltrates leaves with the cell's velocity (reading: q scales with h).
// `r` is the step's rain intensity r(t); cell s takes r w_s.
template <class T>
inline void rain_infiltration(const orc_params& p, double dt, double r, size_t s, T& h,
                              T& qx, T& qy, T* vinf) {
    const double rate = p.rain_w ? r * p.rain_w[s] : r;
    h = h + T(dt) * T(rate);
    if (!p.infil_on) return;
    const double ks = p.ks_f ? p.ks_f[s] : p.ks;
    const double psi = p.psi_f ? p.psi_f[s] : p.psi;
    const double dtheta = p.dtheta_f ? p.dtheta_f[s] : p.dtheta;
    T d;
    if (*vinf > T(0.0)) {
        T zf = *vinf / T(dtheta);                             // Z_f = V_inf / (theta_s - theta_i)
        T ic = T(ks) * (T(1.0) + (T(psi) + h) / zf);          // I_C
        d = vmin(h, T(dt) * ic);                              // dt I = min(h_over, dt I_C)
    } else {
        d = h;  // Z_f = 0: unbounded capacity, all available water infiltrates
    }
    T h_old = h;
    h = h - d;
    *vinf = *vinf + d;  // V_inf^{n+1} = V_inf^n + dt I^n
    if (h_old > T(0.0)) {
        T r = h / h_old;
        qx = qx * r;
        qy = qy * r;
    }
}

// One full time step from time t with a given dt (Algorithm 1: two stages,
// then Heun; at first order one stage, the explicit Euler step).
template <class T>
void step_fixed(const orc_params& p, const T* fric, double t, double dt, T* h, T* qx,
                T* qy, const double* z, T* vinf) {
    size_t n = (size_t)p.nx * p.ny;
    const double r = rain_rate(p, t);
    std::vector<T> h1(n), qx1(n), qy1(n), h2(n), qx2(n), qy2(n);
    stage(p, fric, dt, h, qx, qy, z, h1.data(), qx1.data(), qy1.data(), nullptr);
    if (p.order == 1) {
        for (size_t s = 0; s < n; ++s) {
            T hn = h1[s], qxn = qx1[s], qyn = qy1[s];
            T vdummy = T(0.0);
            rain_infiltration(p, dt, r, s, hn, qxn, qyn, vinf ? &vinf[s] : &vdummy);
            h[s] = hn;
            qx[s] = qxn;
            qy[s] = qyn;
        }
        return;
    }
    stage(p, fric, dt, h1.data(), qx1.data(), qy1.data(), z, h2.data(), qx2.data(),
          qy2.data(), nullptr);
    for (size_t s = 0; s < n; ++s) {
        // U^{n+1} = (U^n + U**)/2
        T hn = T(0.5) * (h[s] + h2[s]);
        T qxn = T(0.5) * (qx[s] + qx2[s]);
        T qyn = T(0.5) * (qy[s] + qy2[s]);
        T vdummy = T(0.0);
        rain_infiltration(p, dt, r, s, hn, qxn, qyn, vinf ? &vinf[s] : &vdummy);
        h[s] = hn;
        qx[s] = qxn;
        qy[s] = qyn;
    }
}

int check_state(size_t n, const double* h, const double* qx, const double* qy) {
    int flags = 0;
    for (size_t s = 0; s < n; ++s) {
        if (!std::isfinite(h[s]) || !std::isfinite(qx[s]) || !std::isfinite(qy[s]))
            flags |= 2;
        else if (h[s] < 0.0)
            flags |= 1;
    }
    return flags;
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface used by the tests (host pointers, [ny][nx] row-major FP64)
// ---------------------------------------------------------------------------

extern "C" {

// Status codes: 0 = a step was taken; 1 = t_end already reached (no step);
// -1 = invalid argument; -3 = negative depth; -4 = non-finite value;
// -5 = the time step collapsed below dt_min; -7 = non-finite time step.
int orc_rate(const orc_params* p, const double* h, const double* qx,
             const double* qy, const double* z, double* ph, double* pqx,
             double* pqy, double* amax) {
    if (!p || p->nx < 1 || p->ny < 1) return -1;
    rate<double>(*p, h, qx, qy, z, ph, pqx, pqy, amax);
    return 0;
}

int orc_stage(const orc_params* p, const double* fric, double dt,
              const double* h, const double* qx, const double* qy,
              const double* z, double* ho, double* qxo, double* qyo,
              double* amax) {
    if (!p || p->nx < 1 || p->ny < 1) return -1;
    stage<double>(*p, fric, dt, h, qx, qy, z, ho, qxo, qyo, amax);
    return 0;
}

double orc_time_step(const orc_params* p, const double* amax, double t,
                     double t_end) {
    return time_step(*p, amax, t, t_end);
}

// Advance up to nsteps steps (stopping at t_end).  dt_log (may be NULL)
// receives each step's dt.  *done receives the number of steps taken.
int orc_run(const orc_params* p, double* h, double* qx, double* qy,
            const double* z, const double* fric, double* vinf, double* t,
            double t_end, int32_t nsteps, double* dt_log, int32_t* done) {
    if (!p || p->nx < 1 || p->ny < 1) return -1;
    size_t n = (size_t)p->nx * p->ny;
    std::vector<double> ph(n), pqx(n), pqy(n);
    int32_t k = 0;
    int rc = 0;
    for (; k < nsteps; ++k) {
        double amax[2];
        rate<double>(*p, h, qx, qy, z, ph.data(), pqx.data(), pqy.data(), amax);
        double dt = time_step(*p, amax, *t, t_end);
        if (!std::isfinite(dt)) { rc = -7; break; }
        if (!(dt > 0.0)) { rc = 1; break; }
        if (dt < p->dt_min && dt < t_end - *t) { rc = -5; break; }
        step_fixed<double>(*p, fric, *t, dt, h, qx, qy, z, vinf);
        *t = *t + dt;
        if (dt_log) dt_log[k] = dt;
        int f = check_state(n, h, qx, qy);
        if (f & 2) { ++k; rc = -4; break; }
        if (f & 1) { ++k; rc = -3; break; }
    }
    if (done) *done = k;
    return rc;
}

// One step from time t with an imposed dt (used for windowed checks of
// large grids).
int orc_step_fixed(const orc_params* p, double t, double dt, double* h, double* qx,
                   double* qy, const double* z, const double* fric,
                   double* vinf) {
    if (!p || p->nx < 1 || p->ny < 1) return -1;
    step_fixed<double>(*p, fric, t, dt, h, qx, qy, z, vinf);
    return 0;
}

// --- single-formula entry points for the unit pins -------------------------

double orc_minmod(double a, double b) { return minmod(a, b); }

// threads the parallel loops use
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

// set the number of threads of the parallel loops (results do not depend on
// it: every cell is computed alone and the maxima are exact)
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

// prim rows: {h, un, ut, eta} for cells i-1, i, i+1.  out: {h_m, h_p, z_m,
// z_p, un_m, un_p, ut_m, ut_p}.
void orc_muscl(const double* a, const double* c, const double* b,
               double h_eps, double* out) {
    Prim<double> pa{a[0], a[1], a[2], a[3]}, pc{c[0], c[1], c[2], c[3]},
        pb{b[0], b[1], b[2], b[3]};
    Recon<double> r = muscl(pa, pc, pb, h_eps);
    double o[8] = {r.h_m, r.h_p, r.z_m, r.z_p, r.un_m, r.un_p, r.ut_m, r.ut_p};
    std::memcpy(out, o, sizeof o);
}

// The same for the ENO reconstructions (modified != 0: modified ENO).
void orc_eno(const double* a, const double* c, const double* b, double h_eps, int modified,
             double* out) {
    Prim<double> pa{a[0], a[1], a[2], a[3]}, pc{c[0], c[1], c[2], c[3]},
        pb{b[0], b[1], b[2], b[3]};
    Recon<double> r = eno(pa, pc, pb, h_eps, modified != 0);
    double o[8] = {r.h_m, r.h_p, r.z_m, r.z_p, r.un_m, r.un_p, r.ut_m, r.ut_p};
    std::memcpy(out, o, sizeof o);
}

void orc_hll(double g, double hL, double unL, double utL, double hR,
             double unR, double utR, double* F) {
    hll(g, hL, unL, utL, hR, unR, utR, F);
}

// out: {F0, F1, F2, sL, sR, speed}
void orc_face(double g, double hm, double zm, double unm, double utm,
              double hp, double zp, double unp, double utp, double* out, int32_t flux) {
    Face<double> f = face(g, hm, zm, unm, utm, hp, zp, unp, utp, flux);
    out[0] = f.F[0]; out[1] = f.F[1]; out[2] = f.F[2];
    out[3] = f.sL; out[4] = f.sR; out[5] = f.speed;
}

// --- tangent (forward-mode) run for the adjoint pin ------------------------
//
// Runs nsteps steps with the imposed dt sequence dts[] (the time steps are
// frozen), propagating a directional derivative with respect to the friction
// field in direction dfric.  The loss is
//   L = sum over k with (k+1) % every == 0, over gauges m, of
//       (h_k[gauge_m] - obs[k/every][m])^2,
// evaluated after step k.  Returns L in *loss and dL (along dfric) in *dloss.
int orc_tangent_run(const orc_params* p, const double* h0, const double* qx0,
                    const double* qy0, const double* z, const double* fric,
                    const double* dfric, int32_t nsteps, const double* dts,
                    const int32_t* gauges, int32_t ngauges, int32_t every,
                    const double* obs, double* loss, double* dloss) {
    if (!p || p->nx < 1 || p->ny < 1 || !fric) return -1;
    size_t n = (size_t)p->nx * p->ny;
    std::vector<Dual> h(n), qx(n), qy(n), fr(n);
    for (size_t s = 0; s < n; ++s) {
        h[s] = Dual(h0[s]);
        qx[s] = Dual(qx0[s]);
        qy[s] = Dual(qy0[s]);
        fr[s] = Dual(fric[s], dfric ? dfric[s] : 0.0);
    }
    Dual L(0.0);
    int obs_row = 0;
    double t = 0.0;
    for (int32_t k = 0; k < nsteps; ++k) {
        step_fixed<Dual>(*p, fr.data(), t, dts[k], h.data(), qx.data(), qy.data(), z,
                         nullptr);
        t = t + dts[k];
        if (every > 0 && (k + 1) % every == 0) {
            for (int32_t m = 0; m < ngauges; ++m) {
                Dual e = h[gauges[m]] - Dual(obs[(size_t)obs_row * ngauges + m]);
                L = L + e * e;
            }
            ++obs_row;
        }
    }
    *loss = L.v;
    *dloss = L.d;
    return 0;
}

// Gauge depths after every `every` steps with an imposed dt sequence (plain
// double; used to build synthetic observations and the loss).
int orc_gauge_run(const orc_params* p, double* h, double* qx, double* qy,
                  const double* z, const double* fric, int32_t nsteps,
                  const double* dts, const int32_t* gauges, int32_t ngauges,
                  int32_t every, double* out) {
    if (!p || p->nx < 1 || p->ny < 1) return -1;
    int row = 0;
    double t = 0.0;
    for (int32_t k = 0; k < nsteps; ++k) {
        step_fixed<double>(*p, fric, t, dts[k], h, qx, qy, z, nullptr);
        t = t + dts[k];
        if (every > 0 && (k + 1) % every == 0) {
            for (int32_t m = 0; m < ngauges; ++m)
                out[(size_t)row * ngauges + m] = h[gauges[m]];
            ++row;
        }
    }
    return 0;
}

}  // extern "C"
