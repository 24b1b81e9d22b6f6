// Host-side helpers shared by the single-simulation context and the
// ensemble: parameter validation, kernel parameter packing, launch shapes,
// the kernels that do not belong to a stage, and the launch of one stage
// for a given strip width.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "swe.h"
#include "swe_device.h"

namespace swe_host {

using namespace swe_dev;

inline size_t ncells(const swe_params* p) { return (size_t)p->nx * (size_t)p->ny; }

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// The imposed values of a side of type `type`: a depth finite and > 0 where
// it is imposed, a discharge finite and >= 0 where it is imposed.
inline bool imposed_values_ok(int type, double h_b, double q_b) {
    if (type == SWE_BC_IMPOSED_H || type == SWE_BC_IMPOSED_HQ)
        if (!(h_b > 0.0) || !std::isfinite(h_b)) return false;
    if (type == SWE_BC_IMPOSED_Q || type == SWE_BC_IMPOSED_HQ)
        if (!(q_b >= 0.0) || !std::isfinite(q_b)) return false;
    return true;
}

inline int check_params(const swe_params* p) {
    if (!p) return SWE_EINVAL;
    if (p->nx < 2 || p->ny < 2) return SWE_EINVAL;
    // the tile kernels address a cell as its row plus a 32-bit byte offset
    if (p->nx > SWE_MAX_NX) return SWE_EINVAL;
    if (!(p->dx > 0.0) || !(p->dy > 0.0) || !(p->g > 0.0) || !(p->cfl > 0.0))
        return SWE_EINVAL;
    if (!(p->h_eps >= 0.0) || !(p->dt_max > 0.0)) return SWE_EINVAL;
    if (!(p->dt_min >= 0.0) || !std::isfinite(p->dt_min)) return SWE_EINVAL;
    for (int k = 0; k < 4; ++k) {
        if (p->bc[k] < SWE_BC_WALL || p->bc[k] > SWE_BC_IMPOSED_HQ) return SWE_EINVAL;
        if (!imposed_values_ok(p->bc[k], p->bc_h[k], p->bc_q[k])) return SWE_EINVAL;
    }
    if (p->fric_law < SWE_FRIC_NONE || p->fric_law > SWE_FRIC_DARCY) return SWE_EINVAL;
    if (p->infil_on && !(p->dtheta > 0.0)) return SWE_EINVAL;
    if (!(p->rain >= 0.0) || !std::isfinite(p->rain)) return SWE_EINVAL;
    if ((size_t)p->nx * (size_t)p->ny > ((size_t)1 << 36)) return SWE_EINVAL;
    if (p->order < 0 || p->order > 2) return SWE_EINVAL;
    if (p->flux < 0 || p->flux > 3) return SWE_EINVAL;
    if (p->recon < 0 || p->recon > 2) return SWE_EINVAL;
    return SWE_OK;
}

// v = 2^k with a normal inverse: inv = 2^-k, and x / v == x * inv for every x
inline bool exact_pow2(double v, double& inv) {
    int e = 0;
    double m = std::frexp(v, &e);
    if (!(v > 0.0) || m != 0.5) return false;
    inv = std::ldexp(1.0, 1 - e);
    return std::isnormal(inv);
}

inline KParams to_kparams(const swe_params& p) {
    KParams k;
    k.nx = p.nx; k.ny = p.ny;
    k.dx = p.dx; k.dy = p.dy; k.g = p.g; k.cfl = p.cfl; k.dt_max = p.dt_max;
    k.dt_min = p.dt_min;
    k.h_eps = p.h_eps;
    k.bcw = p.bc[0]; k.bce = p.bc[1]; k.bcs = p.bc[2]; k.bcn = p.bc[3];
    k.imposed = 0;
    for (int s = 0; s < 4; ++s) {
        k.bc_h[s] = p.bc_h[s];
        k.bc_q[s] = p.bc_q[s];
        if (p.bc[s] >= SWE_BC_IMPOSED_H) k.imposed = 1;
    }
    k.law = p.fric_law; k.coef = p.fric_coef; k.rain = p.rain;
    k.infil = p.infil_on; k.ks = p.ks; k.psi = p.psi; k.dtheta = p.dtheta;
    k.order = p.order == 1 ? 1 : 2;
    k.recon = p.order == 1 ? 0 : p.recon;
    k.flux = p.flux;
    double ix = 0.0, iy = 0.0;
    k.dxy_pow2 = exact_pow2(p.dx, ix) && exact_pow2(p.dy, iy);
    k.inv_dx = k.dxy_pow2 ? ix : 0.0;
    k.inv_dy = k.dxy_pow2 ? iy : 0.0;
    auto in = [](double v, double lo, double hi) { return v >= lo && v <= hi; };
    k.fast_div = in(p.g, 0x1p-1074, 0x1p10) && in(p.dx, 0x1p-300, 0x1p300) &&
                 in(p.dy, 0x1p-300, 0x1p300);
    return k;
}

inline bool valid_tx(int tx) { return tx == 64 || tx == 128 || tx == 256; }

// ORDER template argument of the tile routine for a simulation: 1 first
// order, 2 MUSCL, 3 ENO, 4 modified ENO
inline int order_code(const KParams& p) { return p.order == 1 ? 1 : 2 + p.recon; }

// Default strip width: one-wave strips (no LDS, no barrier) below 8M cells,
// where they give enough blocks to fill the GPU; 256-column strips above
// (less halo work per output column).
inline int default_tx(int nx, int ny) { return (long long)nx * ny < (8LL << 20) ? 64 : 256; }

inline int strips_of(int nx, int tx) {
    int outw = tx - 2 * HALO;
    return (nx + outw - 1) / outw;
}

// Rows per tile: enough tiles to fill 256 CUs many times over (a short last
// wave of tiles), at most 64 rows (each tile re-reads two halo rows above
// and below).
inline int auto_rows(int nx, int ny, int tx) {
    long long strips = strips_of(nx, tx);
    long long ty = (strips * (long long)ny) / 8192;
    if (ty > 64) ty = 64;
    if (ty < 8) ty = 8;
    // keep the grid's y dimension within the launch limit
    while ((ny + ty - 1) / ty > 65535) ty *= 2;
    return (int)ty;
}

inline int hip_ok(hipError_t e) { return e == hipSuccess ? SWE_OK : SWE_EHIP; }

// A roctx range over the host work of an entry point (the enqueueing of a
// step sequence, a forward or reverse adjoint pass), seen by rocprofv3
// --marker-trace beside the kernels it launched.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

// Host mirror of step_io(): the buffers of one step.
inline TileIO host_step_io(const MemberArgs& m, int phase, int slot, double t_end) {
    TileIO io;
    std::memset(&io, 0, sizeof io);
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
    return io;
}

// A validated hyetograph laid out like the tail of the scalar block
// (hy_n, hy_pad, hy_t, hy_r), for one host-to-device copy.
struct HyetoStage {
    int n;
    int pad;
    double t[SWE_HYETO_MAX];
    double r[SWE_HYETO_MAX];
};
static_assert(offsetof(DevScalars, hy_t) - offsetof(DevScalars, hy_n) == offsetof(HyetoStage, t) &&
                  offsetof(DevScalars, hy_r) - offsetof(DevScalars, hy_n) == offsetof(HyetoStage, r),
              "hyetograph staging layout");

inline int stage_hyetograph(const double* t, const double* r, int32_t n, HyetoStage& st) {
    if (n < 0 || n > SWE_HYETO_MAX) return SWE_EINVAL;
    if (n > 0 && (!t || !r)) return SWE_EINVAL;
    std::memset(&st, 0, sizeof st);
    st.n = n;
    for (int k = 0; k < n; ++k) {
        if (!std::isfinite(t[k]) || !std::isfinite(r[k]) || !(r[k] >= 0.0)) return SWE_EINVAL;
        if (k > 0 && !(t[k] > t[k - 1])) return SWE_EINVAL;
        st.t[k] = t[k];
        st.r[k] = r[k];
    }
    return SWE_OK;
}

// Stream-ordered copy into a scalar block; waits for it, so the host table
// may be reused on return.
inline int upload_hyetograph(DevScalars* sc, const HyetoStage& st, hipStream_t s) {
    if (hipMemcpyAsync(&sc->hy_n, &st, sizeof st, hipMemcpyHostToDevice, s) != hipSuccess)
        return SWE_EHIP;
    return hipStreamSynchronize(s) == hipSuccess ? SWE_OK : SWE_EHIP;
}

// The optional per-cell fields of a buffer set.
inline void attach_fields(MemberArgs& m, const swe_buffers& b) {
    m.rain_w = b.rain_w;
    m.ks_f = b.ks;
    m.psi_f = b.psi;
    m.dth_f = b.dtheta;
}

}  // namespace swe_host

// Kernels that are not stages.  Internal linkage: each translation unit
// that includes this header gets its own copy.
static __global__ void swe_init_scalars_kernel(swe_dev::DevScalars* sc, double t) {
    if (blockIdx.x == 0 && threadIdx.x < swe_dev::AMAX_SPREAD)
        for (int s = 0; s < 3; ++s) {
            sc->amax[s][threadIdx.x][0] = 0ull;
            sc->amax[s][threadIdx.x][1] = 0ull;
        }
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc->t[0] = t;
        sc->t[1] = t;
        sc->steps[0] = 0;
        sc->steps[1] = 0;
        sc->last_dt = 0.0;
        sc->status = 0u;
        sc->rain_depth = 0.0;
        sc->water0 = 0.0;
        sc->hy_n = 0;
    }
}

static __global__ void swe_set_time_kernel(swe_dev::DevScalars* sc, int slot, double t) {
    if (threadIdx.x == 0 && blockIdx.x == 0) sc->t[slot] = t;
}

static __global__ void swe_clear_amax_kernel(swe_dev::DevScalars* sc, int slot) {
    if (blockIdx.x == 0 && threadIdx.x < swe_dev::AMAX_SPREAD) {
        sc->amax[slot][threadIdx.x][0] = 0ull;
        sc->amax[slot][threadIdx.x][1] = 0ull;
    }
}

static __global__ void swe_copy_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                       size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = src[i];
}
