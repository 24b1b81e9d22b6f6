// Single-simulation context and its C ABI (include/swe.h) for the
// well-balanced 2D Saint-Venant step on MI355X (gfx950).
//
// Method: arXiv:1307.4839, Sections 2-3.  One time step is two launches of
// the tile routine of swe_device.h over a grid of (strip, row range) tiles:
//
//   stage 1 (rate):   reads U^n and z, writes the convective rate Phi(U^n)
//                     of eq. (SW1Dscheme) extended to 2D by the method of
//                     lines, and max-reduces the face wave-speed bounds of
//                     eq. (cfl) on the device;
//   stage 2 (update): derives dt from the bounds, rebuilds
//                     U* = friction(U^n + dt Phi(U^n)) on the fly, evaluates
//                     Phi(U*), U** = friction(U* + dt Phi(U*)), Heun's average
//                     (Section 3.2), rain and Green-Ampt (Section 3.5), and
//                     writes U^{n+1}.
//
// HBM traffic per cell and step: stage 1 reads 32 B and writes 24 B; stage 2
// reads 56 B (+8 B with a friction field, +8 B V_inf) and writes 24 B
// (+8 B V_inf).  Face values never go to HBM.  Time, step count and the
// wave-speed accumulators live on the device, double-buffered by step
// parity, so a sequence of steps needs no host synchronization; runs of 16
// steps are replayed from a captured HIP graph.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "swe.h"
#include "swe_device.h"
#include "swe_host.h"

using namespace swe_dev;
using namespace swe_host;

namespace {

constexpr int DIAG_BLOCKS = 512;  // blocks of the diagnostics reduction
constexpr int DIAG_T = 256;
constexpr int GRAPH_STEPS = 16;   // steps per captured graph (even)

template <int STAGE, int TXT, bool FIELDS, int ORDER, int FLUX>
__global__ __launch_bounds__(TXT) void stage_kernel(MemberArgs m, TileIO io, int ty) {
    const int y0 = blockIdx.y * ty;
    const int y1 = min(y0 + ty, m.p.ny);
    stage_tile<STAGE, TXT, FIELDS, ORDER, FLUX>(m, io, blockIdx.x, y0, y1,
                                                blockIdx.x == 0 && blockIdx.y == 0,
                                                blockIdx.x + blockIdx.y * gridDim.x);
}

// First-order update (one Euler stage), cell by cell over a grid-stride loop.
constexpr int EULER_T = 256;
template <bool FIELDS>
__global__ __launch_bounds__(EULER_T) void euler_kernel(MemberArgs m, TileIO io) {
    euler_cells<FIELDS>(m, io, blockIdx.x == 0,
                        (size_t)blockIdx.x * EULER_T + threadIdx.x,
                        (size_t)gridDim.x * EULER_T);
}

// Deterministic diagnostics: block b reduces the cells b, b + B, b + 2B, ...
// in a fixed tree; a single block then combines the partials in order.
// Also sums the rain weight (1 per cell without a weight field).
constexpr int DIAG_N = 6;  // values per block: mass, V_inf, min, max, wet, weight
__global__ __launch_bounds__(DIAG_T) void diag_partial_kernel(
    const double* __restrict__ h, const double* __restrict__ vinf,
    const double* __restrict__ rain_w, double h_eps, size_t n, double* __restrict__ part) {
    __shared__ double s_m[DIAG_T], s_v[DIAG_T], s_lo[DIAG_T], s_hi[DIAG_T], s_w[DIAG_T],
        s_r[DIAG_T];
    double m = 0.0, v = 0.0, lo = INFINITY, hi = -INFINITY, w = 0.0, r = 0.0;
    for (size_t i = (size_t)blockIdx.x * DIAG_T + threadIdx.x; i < n;
         i += (size_t)gridDim.x * DIAG_T) {
        double x = h[i];
        m += x;
        if (vinf) v += vinf[i];
        lo = fmin(lo, x);
        hi = fmax(hi, x);
        if (x > h_eps) w += 1.0;
        r += rain_w ? rain_w[i] : 1.0;
    }
    int t = threadIdx.x;
    s_m[t] = m; s_v[t] = v; s_lo[t] = lo; s_hi[t] = hi; s_w[t] = w; s_r[t] = r;
    __syncthreads();
    for (int off = DIAG_T / 2; off > 0; off >>= 1) {
        if (t < off) {
            s_m[t] += s_m[t + off];
            s_v[t] += s_v[t + off];
            s_lo[t] = fmin(s_lo[t], s_lo[t + off]);
            s_hi[t] = fmax(s_hi[t], s_hi[t + off]);
            s_w[t] += s_w[t + off];
            s_r[t] += s_r[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        double* o = part + (size_t)blockIdx.x * DIAG_N;
        o[0] = s_m[0]; o[1] = s_v[0]; o[2] = s_lo[0]; o[3] = s_hi[0]; o[4] = s_w[0];
        o[5] = s_r[0];
    }
}

// Combines the partials in block order; with `sc`, also keeps the initial
// water (h + V_inf) in the scalar block (the reference of the outflow).
__global__ void diag_final_kernel(double* part, int nb, DevScalars* sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double m = 0.0, v = 0.0, lo = INFINITY, hi = -INFINITY, w = 0.0, r = 0.0;
        for (int b = 0; b < nb; ++b) {
            const double* o = part + (size_t)b * DIAG_N;
            m += o[0]; v += o[1]; lo = fmin(lo, o[2]); hi = fmax(hi, o[3]); w += o[4];
            r += o[5];
        }
        part[0] = m; part[1] = v; part[2] = lo; part[3] = hi; part[4] = w; part[5] = r;
        if (sc) sc->water0 = m + v;
    }
}

template <int STAGE, bool FIELDS, int ORDER, int FLUX>
void launch_stage_tf(int tx, dim3 grid, hipStream_t s, const MemberArgs& m, const TileIO& io,
                     int ty) {
    switch (tx) {
        case 64: hipLaunchKernelGGL((stage_kernel<STAGE, 64, FIELDS, ORDER, FLUX>), grid, dim3(64), 0, s, m, io, ty); break;
        case 128: hipLaunchKernelGGL((stage_kernel<STAGE, 128, FIELDS, ORDER, FLUX>), grid, dim3(128), 0, s, m, io, ty); break;
        default: hipLaunchKernelGGL((stage_kernel<STAGE, 256, FIELDS, ORDER, FLUX>), grid, dim3(256), 0, s, m, io, ty); break;
    }
}

template <int STAGE, bool FIELDS, int ORDER>
void launch_stage_t(int tx, dim3 grid, hipStream_t s, const MemberArgs& m, const TileIO& io,
                    int ty) {
    if (m.p.flux == 3)
        launch_stage_tf<STAGE, FIELDS, ORDER, 3>(tx, grid, s, m, io, ty);
    else if (m.p.flux == 2)
        launch_stage_tf<STAGE, FIELDS, ORDER, 2>(tx, grid, s, m, io, ty);
    else if (m.p.flux == 1)
        launch_stage_tf<STAGE, FIELDS, ORDER, 1>(tx, grid, s, m, io, ty);
    else
        launch_stage_tf<STAGE, FIELDS, ORDER, 0>(tx, grid, s, m, io, ty);
}

template <int STAGE, bool FIELDS>
void launch_stage_o(int tx, dim3 grid, hipStream_t s, const MemberArgs& m, const TileIO& io,
                    int ty) {
    switch (order_code(m.p)) {
        case 1:
            if constexpr (STAGE == 1) launch_stage_t<1, FIELDS, 1>(tx, grid, s, m, io, ty);
            break;
        case 3: launch_stage_t<STAGE, FIELDS, 3>(tx, grid, s, m, io, ty); break;
        case 4: launch_stage_t<STAGE, FIELDS, 4>(tx, grid, s, m, io, ty); break;
        default: launch_stage_t<STAGE, FIELDS, 2>(tx, grid, s, m, io, ty); break;
    }
}

// Stage 1 never reads the rain and soil fields: its FIELDS variant only
// adds the ghosts of imposed sides.  The first-order scheme has only stage 1
// (its update is euler_kernel).
template <int STAGE>
void launch_stage(int tx, dim3 grid, hipStream_t s, const MemberArgs& m, const TileIO& io,
                  int ty) {
    const bool fields = STAGE == 1 ? m.p.imposed != 0 : (has_fields(m) || m.p.imposed);
    if (fields)
        launch_stage_o<STAGE, true>(tx, grid, s, m, io, ty);
    else
        launch_stage_o<STAGE, false>(tx, grid, s, m, io, ty);
}

void launch_euler(hipStream_t s, const MemberArgs& m, const TileIO& io) {
    const size_t n = (size_t)m.p.nx * (size_t)m.p.ny;
    const unsigned blocks = (unsigned)std::min<size_t>((n + EULER_T - 1) / EULER_T, 16384);
    if (has_fields(m))
        hipLaunchKernelGGL(euler_kernel<true>, dim3(blocks), dim3(EULER_T), 0, s, m, io);
    else
        hipLaunchKernelGGL(euler_kernel<false>, dim3(blocks), dim3(EULER_T), 0, s, m, io);
}

}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------

struct swe_ctx {
    swe_params prm;
    MemberArgs m;       // kernel view of the simulation
    hipStream_t stream;
    double* diag;       // diagnostics partials
    int slot;           // parity of the next step
    int tx, ty;         // strip width (threads per block) and rows per tile
    // captured GRAPH_STEPS-step sequence, valid for (slot, t_end, epoch)
    hipGraphExec_t graph;
    hipStream_t cap_stream;  // private stream used only to capture graphs
    int graph_slot;
    double graph_t_end;
    unsigned graph_epoch;
    unsigned epoch;     // bumped whenever a baked-in kernel argument changes
    // optional per-kernel timing: events before stage 1, between the
    // stages and after stage 2 of each profiled step
    hipEvent_t* prof_ev;
    int prof_cap;
    int prof_n;
    // gauge recorder (caller-owned device arrays); g_n = 0: off
    const int32_t* g_cells;
    int32_t g_n;
    int32_t g_every;
    double* g_series;
    int64_t g_cap;
    long long g_base;  // step count when the gauges were set
};

namespace {

constexpr int GAUGE_T = 256;

// Gauge samples after a step that read slot `slot`: the step advanced the
// simulation when steps[slot ^ 1] (its count after) differs from
// steps[slot] (before).  A count d = after - base that is a positive
// multiple of `every` records sample k = d / every - 1 of h (the step's
// output) at every gauge, while k < cap; a cell outside the grid records NaN.
__global__ __launch_bounds__(GAUGE_T) void gauge_record_kernel(
    const double* __restrict__ h, const int32_t* __restrict__ cells, int n, int every,
    double* __restrict__ series, long long cap, const DevScalars* __restrict__ sc, int slot,
    long long base, long long ncell) {
    const long long after = sc->steps[slot ^ 1];
    if (after == sc->steps[slot]) return;
    const long long d = after - base;
    if (d <= 0 || d % every != 0) return;
    const long long k = d / every - 1;
    if (k >= cap) return;
    const int g = blockIdx.x * GAUGE_T + threadIdx.x;
    if (g >= n) return;
    const long long cell = cells[g];
    series[k * n + g] = (cell >= 0 && cell < ncell) ? h[cell] : __builtin_nan("");
}

dim3 stage_grid(const swe_ctx* c) {
    return dim3(strips_of(c->prm.nx, c->tx), (c->prm.ny + c->ty - 1) / c->ty);
}

// Enqueue one step reading state buffer `phase` (0 = caller's, 1 = workspace).
void enqueue_step(swe_ctx* c, int phase, double t_end, bool profile) {
    TileIO io = host_step_io(c->m, phase, c->slot, t_end);
    dim3 grid = stage_grid(c);
    bool prof = profile && c->prof_ev && c->prof_n < c->prof_cap;
    if (prof) (void)hipEventRecord(c->prof_ev[3 * c->prof_n], c->stream);
    launch_stage<1>(c->tx, grid, c->stream, c->m, io, c->ty);
    if (prof) (void)hipEventRecord(c->prof_ev[3 * c->prof_n + 1], c->stream);
    if (c->m.p.order == 1)
        launch_euler(c->stream, c->m, io);
    else
        launch_stage<2>(c->tx, grid, c->stream, c->m, io, c->ty);
    if (prof) (void)hipEventRecord(c->prof_ev[3 * c->prof_n++ + 2], c->stream);
    if (c->g_n > 0)
        hipLaunchKernelGGL(gauge_record_kernel, dim3((c->g_n + GAUGE_T - 1) / GAUGE_T),
                           dim3(GAUGE_T), 0, c->stream, (const double*)io.ho, c->g_cells, c->g_n,
                           c->g_every, c->g_series, (long long)c->g_cap,
                           (const DevScalars*)c->m.sc, c->slot, c->g_base,
                           (long long)ncells(&c->prm));
    c->slot ^= 1;
}

void drop_graph(swe_ctx* c) {
    if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
}

// Capture GRAPH_STEPS steps (an even number, so the state buffer and the
// slot return to where they started) on the context stream.
int ensure_graph(swe_ctx* c, double t_end) {
    if (c->graph && c->graph_slot == c->slot && c->graph_t_end == t_end &&
        c->graph_epoch == c->epoch)
        return SWE_OK;
    drop_graph(c);
    int slot0 = c->slot;
    // the caller's stream may be the legacy default stream, which cannot be
    // captured: record on a private stream, launch on the caller's
    if (!c->cap_stream &&
        hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        c->cap_stream = nullptr;
        return SWE_EHIP;
    }
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        c->stream = user;
        return SWE_EHIP;
    }
    for (int k = 0; k < GRAPH_STEPS; ++k) enqueue_step(c, k & 1, t_end, false);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    c->stream = user;
    c->slot = slot0;
    if (e != hipSuccess || !g) return SWE_EHIP;
    e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->graph = nullptr;
        return SWE_EHIP;
    }
    c->graph_slot = slot0;
    c->graph_t_end = t_end;
    c->graph_epoch = c->epoch;
    return SWE_OK;
}

}  // namespace

extern "C" {

int swe_workspace_bytes(const swe_params* p, size_t* bytes) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!bytes) return SWE_EINVAL;
    size_t n = ncells(p);
    *bytes = SCALAR_BYTES + 6 * align256(n * sizeof(double)) +
             align256((size_t)DIAG_BLOCKS * DIAG_N * sizeof(double));
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
    c->stream = (hipStream_t)stream;
    char* w = (char*)workspace;
    size_t n = ncells(p), an = align256(n * sizeof(double));
    MemberArgs& m = c->m;
    m.p = to_kparams(*p);
    m.z = b->z;
    m.fric = b->fric;
    m.vinf = p->infil_on ? b->vinf : nullptr;
    attach_fields(m, *b);
    m.sc = (DevScalars*)w;
    w += SCALAR_BYTES;
    m.h[0] = b->h; m.qx[0] = b->qx; m.qy[0] = b->qy;
    m.h[1] = (double*)w; w += an;
    m.qx[1] = (double*)w; w += an;
    m.qy[1] = (double*)w; w += an;
    m.ph = (double*)w; w += an;
    m.pqx = (double*)w; w += an;
    m.pqy = (double*)w; w += an;
    c->diag = (double*)w;
    c->slot = 0;
    c->tx = default_tx(p->nx, p->ny);
    c->ty = auto_rows(p->nx, p->ny, c->tx);
    hipLaunchKernelGGL(swe_init_scalars_kernel, dim3(1), dim3(64), 0, c->stream, m.sc, 0.0);
    // the initial water, kept on the device for the outflow diagnostic
    hipLaunchKernelGGL(diag_partial_kernel, dim3(DIAG_BLOCKS), dim3(DIAG_T), 0, c->stream,
                       (const double*)m.h[0], (const double*)m.vinf, m.rain_w, p->h_eps, n,
                       c->diag);
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(64), 0, c->stream, c->diag,
                       DIAG_BLOCKS, m.sc);
    rc = hip_ok(hipGetLastError());
    if (rc) { delete c; return rc; }
    *out = c;
    return SWE_OK;
}

int swe_destroy(swe_ctx* c) {
    if (!c) return SWE_OK;
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->prof_ev) {
        for (int k = 0; k < 3 * c->prof_cap; ++k) (void)hipEventDestroy(c->prof_ev[k]);
        delete[] c->prof_ev;
    }
    delete c;
    return SWE_OK;
}

int swe_set_tiling(swe_ctx* c, int32_t tx, int32_t ty) {
    if (!c || !valid_tx(tx) || ty < 0 || ty > c->prm.ny) return SWE_EINVAL;
    if (ty > 0 && (c->prm.ny + ty - 1) / ty > 65535) return SWE_EINVAL;
    c->tx = tx;
    c->ty = ty == 0 ? auto_rows(c->prm.nx, c->prm.ny, tx) : ty;
    c->epoch++;
    return SWE_OK;
}

int swe_get_tiling(swe_ctx* c, int32_t* tx, int32_t* ty) {
    if (!c) return SWE_EINVAL;
    if (tx) *tx = c->tx;
    if (ty) *ty = c->ty;
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
    hipLaunchKernelGGL(swe_set_time_kernel, dim3(1), dim3(64), 0, c->stream, c->m.sc, c->slot, t);
    return hip_ok(hipGetLastError());
}

int swe_set_rain(swe_ctx* c, double rain) {
    if (!c || !(rain >= 0.0) || !std::isfinite(rain)) return SWE_EINVAL;
    c->prm.rain = rain;
    c->m.p.rain = rain;
    c->epoch++;
    return SWE_OK;
}

int swe_set_boundary_values(swe_ctx* c, int32_t side, double h_b, double q_b) {
    if (!c || side < 0 || side > 3) return SWE_EINVAL;
    const int type = c->prm.bc[side];
    if (type < SWE_BC_IMPOSED_H || !imposed_values_ok(type, h_b, q_b)) return SWE_EINVAL;
    c->prm.bc_h[side] = h_b;
    c->prm.bc_q[side] = q_b;
    c->m.p.bc_h[side] = h_b;
    c->m.p.bc_q[side] = q_b;
    c->epoch++;
    return SWE_OK;
}

int swe_set_hyetograph(swe_ctx* c, const double* t_pts, const double* r, int32_t n) {
    if (!c) return SWE_EINVAL;
    HyetoStage st;
    int rc = stage_hyetograph(t_pts, r, n, st);
    if (rc) return rc;
    return upload_hyetograph(c->m.sc, st, c->stream);
}

int swe_set_dt_log(swe_ctx* c, double* dev_log, int64_t capacity) {
    if (!c || capacity < 0) return SWE_EINVAL;
    c->m.dtlog = dev_log;
    c->m.dtlog_cap = dev_log ? capacity : 0;
    c->epoch++;
    return SWE_OK;
}

int swe_set_gauges(swe_ctx* c, const int32_t* cells, int32_t ngauges, int32_t every,
                   double* series, int64_t max_samples) {
    if (!c || ngauges < 0) return SWE_EINVAL;
    if (ngauges > 0 && (!cells || !series || every < 1 || max_samples < 1)) return SWE_EINVAL;
    long long st = 0;
    if (ngauges > 0) {
        if (hipMemcpyAsync(&st, &c->m.sc->steps[c->slot], sizeof st, hipMemcpyDeviceToHost,
                           c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return SWE_EHIP;
    }
    c->g_cells = ngauges > 0 ? cells : nullptr;
    c->g_n = ngauges;
    c->g_every = ngauges > 0 ? every : 1;
    c->g_series = ngauges > 0 ? series : nullptr;
    c->g_cap = ngauges > 0 ? max_samples : 0;
    c->g_base = st;
    c->epoch++;
    return SWE_OK;
}

int swe_get_gauges(swe_ctx* c, double* out, int64_t max_copy, int64_t* nsamples) {
    if (!c || max_copy < 0) return SWE_EINVAL;
    if (c->g_n == 0) {
        if (nsamples) *nsamples = 0;
        return SWE_OK;
    }
    long long st = 0;
    if (hipMemcpyAsync(&st, &c->m.sc->steps[c->slot], sizeof st, hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return SWE_EHIP;
    long long k = (st - c->g_base) / c->g_every;
    if (k > c->g_cap) k = c->g_cap;
    if (k < 0) k = 0;
    if (nsamples) *nsamples = k;
    const long long ncopy = k < max_copy ? k : max_copy;
    if (out && ncopy > 0) {
        if (hipMemcpyAsync(out, c->g_series, (size_t)ncopy * c->g_n * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return SWE_EHIP;
    }
    return SWE_OK;
}

}  // extern "C"

namespace {

// Steps enqueued between two reads of the time when a long run may end
// early (even, a multiple of GRAPH_STEPS).
constexpr int32_t STOP_CHUNK = 256;

int step_run(swe_ctx* c, int32_t nsteps, double t_end) {
    const bool profiling = c->prof_ev != nullptr;
    int32_t k = 0;
    // whole graphs first (not while profiling: events go between kernels)
    if (!profiling && nsteps >= GRAPH_STEPS) {
        int rc = ensure_graph(c, t_end);
        if (rc) return rc;
        for (; k + GRAPH_STEPS <= nsteps; k += GRAPH_STEPS)
            if (hipGraphLaunch(c->graph, c->stream) != hipSuccess) return SWE_EHIP;
    }
    // the rest one by one; the state alternates between the caller's
    // buffers (0) and the workspace copy (1)
    int phase = 0;
    for (; k < nsteps; ++k) {
        enqueue_step(c, phase, t_end, true);
        phase ^= 1;
    }
    if (phase == 1) {
        size_t n = ncells(&c->prm);
        hipLaunchKernelGGL(swe_copy_kernel, dim3(1024), dim3(256), 0, c->stream,
                           (const double*)c->m.h[1], c->m.h[0], n);
        hipLaunchKernelGGL(swe_copy_kernel, dim3(1024), dim3(256), 0, c->stream,
                           (const double*)c->m.qx[1], c->m.qx[0], n);
        hipLaunchKernelGGL(swe_copy_kernel, dim3(1024), dim3(256), 0, c->stream,
                           (const double*)c->m.qy[1], c->m.qy[0], n);
    }
    return hip_ok(hipGetLastError());
}

}  // namespace

extern "C" {

int swe_step(swe_ctx* c, int32_t nsteps, double t_end) {
    if (!c || nsteps < 0 || std::isnan(t_end)) return SWE_EINVAL;
    if (nsteps == 0) return SWE_OK;
    Range range("swe_step");
    if (!std::isfinite(t_end) || nsteps <= STOP_CHUNK) return step_run(c, nsteps, t_end);
    // a finite end time: enqueue chunks and stop once it is reached, instead
    // of enqueueing steps that would all be no-ops
    for (int32_t left = nsteps; left > 0;) {
        const int32_t k = left < STOP_CHUNK ? left : STOP_CHUNK;
        int rc = step_run(c, k, t_end);
        if (rc) return rc;
        left -= k;
        if (left > 0) {
            double t = 0.0;
            if (hipMemcpyAsync(&t, &c->m.sc->t[c->slot], sizeof t, hipMemcpyDeviceToHost,
                               c->stream) != hipSuccess ||
                hipStreamSynchronize(c->stream) != hipSuccess)
                return SWE_EHIP;
            if (t >= t_end) break;
        }
    }
    return SWE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Runs without allocation (swe_run_noalloc)
// ---------------------------------------------------------------------------

namespace {

// A scalar block, a second state and the stage rate for grids of up to
// SWE_NOALLOC_MAX_CELLS cells: the workspace of swe_run_noalloc.  Every
// device the library runs on holds its own copy until the process ends.
constexpr size_t NOALLOC_PLANE = ((size_t)SWE_NOALLOC_MAX_CELLS * sizeof(double) + 255) / 256 * 256;
constexpr size_t NOALLOC_BYTES = SCALAR_BYTES + 6 * NOALLOC_PLANE;
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// Device address of `scratch` on each device, taken once per device with the
// device current (host code must not use the symbol's name as an address).
constexpr int NOALLOC_DEVICES = 64;
void* g_scratch[NOALLOC_DEVICES];
std::mutex g_scratch_mu;

int scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_DEVICES) return SWE_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return SWE_EHIP;
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return SWE_OK;
}

// t, last dt, steps and status flags of the run into the caller's array
__global__ void noalloc_info_kernel(const DevScalars* sc, int slot, double* info) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        info[0] = sc->t[slot];
        info[1] = sc->last_dt;
        info[2] = (double)sc->steps[slot];
        info[3] = (double)sc->status;
    }
}

}  // namespace

extern "C" {

int swe_run_noalloc(const swe_params* p, const swe_buffers* b, double t0, int32_t nsteps,
                    double t_end, void* stream, double* info) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!b || !info || !b->h || !b->qx || !b->qy || !b->z) return SWE_EINVAL;
    if (p->infil_on && !b->vinf) return SWE_EINVAL;
    if (nsteps < 0 || !std::isfinite(t0) || std::isnan(t_end)) return SWE_EINVAL;
    const size_t n = ncells(p);
    if (n > (size_t)SWE_NOALLOC_MAX_CELLS) return SWE_ENOMEM;
    void* base = nullptr;
    rc = scratch_address(&base);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    MemberArgs m;
    std::memset(&m, 0, sizeof m);
    m.p = to_kparams(*p);
    m.z = b->z;
    m.fric = b->fric;
    m.vinf = p->infil_on ? b->vinf : nullptr;
    attach_fields(m, *b);
    char* w = (char*)base;
    m.sc = (DevScalars*)w;
    w += SCALAR_BYTES;
    m.h[0] = b->h; m.qx[0] = b->qx; m.qy[0] = b->qy;
    m.h[1] = (double*)w; w += NOALLOC_PLANE;
    m.qx[1] = (double*)w; w += NOALLOC_PLANE;
    m.qy[1] = (double*)w; w += NOALLOC_PLANE;
    m.ph = (double*)w; w += NOALLOC_PLANE;
    m.pqx = (double*)w; w += NOALLOC_PLANE;
    m.pqy = (double*)w;
    // the scalar block keeps the last call's contents: start from zero
    // accumulators and flags, time t0 and no hyetograph (a kernel, not a
    // memset)
    hipLaunchKernelGGL(swe_init_scalars_kernel, dim3(1), dim3(64), 0, s, m.sc, t0);
    const int tx = default_tx(p->nx, p->ny), ty = auto_rows(p->nx, p->ny, tx);
    const dim3 grid(strips_of(p->nx, tx), (p->ny + ty - 1) / ty);
    int slot = 0, phase = 0;
    for (int32_t k = 0; k < nsteps; ++k) {
        TileIO io = host_step_io(m, phase, slot, t_end);
        launch_stage<1>(tx, grid, s, m, io, ty);
        if (m.p.order == 1)
            launch_euler(s, m, io);
        else
            launch_stage<2>(tx, grid, s, m, io, ty);
        slot ^= 1;
        phase ^= 1;
    }
    if (phase == 1) {
        hipLaunchKernelGGL(swe_copy_kernel, dim3(1024), dim3(256), 0, s, (const double*)m.h[1],
                           m.h[0], n);
        hipLaunchKernelGGL(swe_copy_kernel, dim3(1024), dim3(256), 0, s, (const double*)m.qx[1],
                           m.qx[0], n);
        hipLaunchKernelGGL(swe_copy_kernel, dim3(1024), dim3(256), 0, s, (const double*)m.qy[1],
                           m.qy[0], n);
    }
    hipLaunchKernelGGL(noalloc_info_kernel, dim3(1), dim3(64), 0, s, (const DevScalars*)m.sc,
                       slot, info);
    return hip_ok(hipGetLastError());
}

int swe_get_time(swe_ctx* c, double* t, double* last_dt, int64_t* steps) {
    if (!c) return SWE_EINVAL;
    DevScalars s;
    if (hipMemcpyAsync(&s, c->m.sc, sizeof s, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
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
    if (hipMemcpyAsync(&s, c->m.sc, sizeof s, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return SWE_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SWE_EHIP;
    if (flags) *flags = s.status;
    if (s.status & SWE_FLAG_NONFINITE) return SWE_ENONFINITE;
    if (s.status & SWE_FLAG_NEGDEPTH) return SWE_ENEGDEPTH;
    if (s.status & SWE_FLAG_DT) return SWE_EDT;
    if (s.status & SWE_FLAG_DT_UNDERFLOW) return SWE_EDTMIN;
    return SWE_OK;
}

int swe_get_diagnostics(swe_ctx* c, swe_diag* d) {
    if (!c || !d) return SWE_EINVAL;
    size_t n = ncells(&c->prm);
    hipLaunchKernelGGL(diag_partial_kernel, dim3(DIAG_BLOCKS), dim3(DIAG_T), 0, c->stream,
                       (const double*)c->m.h[0], (const double*)c->m.vinf, c->m.rain_w,
                       c->prm.h_eps, n, c->diag);
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(64), 0, c->stream, c->diag,
                       DIAG_BLOCKS, (DevScalars*)nullptr);
    double r[DIAG_N];
    DevScalars s;
    if (hipMemcpyAsync(r, c->diag, sizeof r, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipMemcpyAsync(&s, c->m.sc, sizeof s, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return SWE_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SWE_EHIP;
    double area = c->prm.dx * c->prm.dy;
    d->mass = r[0] * area;
    d->infiltrated = r[1] * area;
    d->h_min = r[2];
    d->h_max = r[3];
    d->wet_cells = (int64_t)r[4];
    d->rain_in = s.rain_depth * r[5] * area;
    d->outflow = (s.water0 + s.rain_depth * r[5] - (r[0] + r[1])) * area;
    return SWE_OK;
}

int swe_rate(swe_ctx* c, const double* h, const double* qx, const double* qy,
             double* ph, double* pqx, double* pqy, double* amax) {
    if (!c || !h || !qx || !qy || !ph || !pqx || !pqy) return SWE_EINVAL;
    hipLaunchKernelGGL(swe_clear_amax_kernel, dim3(1), dim3(64), 0, c->stream, c->m.sc, 2);
    TileIO io;
    std::memset(&io, 0, sizeof io);
    io.h = h; io.qx = qx; io.qy = qy;
    io.ph = ph; io.pqx = pqx; io.pqy = pqy;
    // slot 2 of the maxima is reserved for this call and is not a step slot
    io.acc = &c->m.sc->amax[2][0][0];
    io.clr = nullptr;
    io.slot = 2;
    launch_stage<1>(c->tx, stage_grid(c), c->stream, c->m, io, c->ty);
    unsigned long long got[AMAX_SPREAD][AMAX_LINE];
    if (hipMemcpyAsync(got, &c->m.sc->amax[2][0][0], sizeof got, hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess)
        return SWE_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SWE_EHIP;
    if (amax) {
        unsigned long long x = 0ull, y = 0ull;
        for (int k = 0; k < AMAX_SPREAD; ++k) {
            x = std::max(x, got[k][0]);
            y = std::max(y, got[k][1]);
        }
        std::memcpy(&amax[0], &x, 8);
        std::memcpy(&amax[1], &y, 8);
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
        case SWE_EDTMIN: return "time step collapsed below dt_min";
        case SWE_ENOMEM: return "workspace too small";
        default: return "unknown error";
    }
}

}  // extern "C"
