// Ensemble of independent simulations of uneven sizes stepped together
// (C ABI swe_batch_*, include/swe.h).
//
// Every member runs the same two stages as a single simulation (the tile
// routine of swe_device.h; the members share the scheme, order and flux, so
// that one kernel serves each stage), with its own grid, parameters, time,
// time step (its own CFL bound, Section 3.3), status flags and buffers.  A
// step of the whole ensemble is ONE launch per stage over a work list of
// (member, strip, row range) tiles, largest members first: one block per
// tile, dispatched in list order.  (A persistent grid sized to the GPU's
// resident capacity, each block walking the list, held 173 VGPRs in stage 2
// and 2 waves per SIMD; one tile per block holds 162 and 3.)  Runs of 16
// steps replay a captured HIP graph.  The tile shape (strip width x rows) is chosen by a measuring
// autotuner that times the candidates on the live state and restores it
// bit for bit afterwards; results never depend on the tile shape.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "swe.h"
#include "swe_device.h"
#include "swe_host.h"

using namespace swe_dev;
using namespace swe_host;

namespace {

constexpr int GRAPH_STEPS = 16;  // steps per captured graph (even)
constexpr int MIN_TY = 4;        // smallest rows per tile the work list is sized for

template <int STAGE, int TXT, bool FIELDS, int ORDER, int FLUX>
__global__ __launch_bounds__(TXT) void batch_stage_kernel(const MemberArgs* __restrict__ ms,
                                                          const int4* __restrict__ tiles,
                                                          int ntiles, int phase, int slot,
                                                          double t_end) {
    const int k = blockIdx.x;
    if (k >= ntiles) return;
    const int4 tl = tiles[k];  // member, strip, first row, end row
    // read in place (uniform loads): a private copy of the record would live
    // in scratch memory, since its buffer pairs are indexed by phase
    const MemberArgs& m = ms[tl.x];
    const TileIO io = step_io(m, phase, slot, t_end);
    stage_tile<STAGE, TXT, FIELDS, ORDER, FLUX>(m, io, tl.y, tl.z, tl.w,
                                                tl.y == 0 && tl.z == 0, k);
}

// Update of the first-order scheme (Section 3.3: one explicit Euler stage,
// U^{n+1} = friction(U^n + dt Phi(U^n)), then rain and Green-Ampt), tile by
// tile over the same work list: the strip's output columns of each row.
// The arithmetic is that of the single-context update (euler_cells).
template <int TXT, bool FIELDS>
__global__ __launch_bounds__(TXT) void batch_euler_kernel(const MemberArgs* __restrict__ ms,
                                                          const int4* __restrict__ tiles,
                                                          int ntiles, int phase, int slot,
                                                          double t_end) {
    constexpr int OUTW = TXT - 2 * HALO;
    {
        const int k = blockIdx.x;
        if (k >= ntiles) return;
        const int4 tl = tiles[k];
        const MemberArgs& m = ms[tl.x];
        const KParams& p = m.p;
        const TileIO io = step_io(m, phase, slot, t_end);
        double dt, rain;
        // every lane takes part (the hyetograph lookup uses wave ballots)
        const bool go = begin_step(m, io, tl.y == 0 && tl.z == 0, dt, rain);
        const int c = tl.y * OUTW + (int)threadIdx.x;
        if ((int)threadIdx.x >= OUTW || c >= p.nx) return;
        for (int j = tl.z; j < tl.w; ++j) {
            const size_t i = (size_t)j * p.nx + c;
            if (!go) {
                io.ho[i] = io.h[i];
                io.qxo[i] = io.qx[i];
                io.qyo[i] = io.qy[i];
                continue;
            }
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
}

// Copy the workspace state (buffer 1) back to the caller's buffers (0) for
// every member: block row y handles member y.
__global__ void batch_copyback_kernel(const MemberArgs* __restrict__ ms) {
    const MemberArgs& m = ms[blockIdx.y];
    size_t n = (size_t)m.p.nx * m.p.ny;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        m.h[0][i] = m.h[1][i];
        m.qx[0][i] = m.qx[1][i];
        m.qy[0][i] = m.qy[1][i];
    }
}

// Save (dir = 0) or restore (dir = 1) each member's state, V_inf and
// scalar block to/from the backup area.
struct Backup {
    double* h;
    double* qx;
    double* qy;
    double* vinf;
    DevScalars* sc;
};

__global__ void batch_backup_kernel(const MemberArgs* __restrict__ ms,
                                    const Backup* __restrict__ bk, int dir) {
    const MemberArgs& m = ms[blockIdx.y];
    const Backup& b = bk[blockIdx.y];
    size_t n = (size_t)m.p.nx * m.p.ny;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        if (dir == 0) {
            b.h[i] = m.h[0][i];
            b.qx[i] = m.qx[0][i];
            b.qy[i] = m.qy[0][i];
            if (m.vinf) b.vinf[i] = m.vinf[i];
        } else {
            m.h[0][i] = b.h[i];
            m.qx[0][i] = b.qx[i];
            m.qy[0][i] = b.qy[i];
            if (m.vinf) m.vinf[i] = b.vinf[i];
        }
    }
    if (blockIdx.x == 0) {
        // the scalar block, word by word across the block's threads
        const unsigned long long* src =
            (const unsigned long long*)(dir == 0 ? (const void*)m.sc : (const void*)b.sc);
        unsigned long long* dst = (unsigned long long*)(dir == 0 ? (void*)b.sc : (void*)m.sc);
        for (size_t i = threadIdx.x; i < sizeof(DevScalars) / 8; i += blockDim.x) dst[i] = src[i];
    }
}

// The scheme of an ensemble (shared by its members) and whether the
// FIELDS variant of the tile routine is needed: some member has a rain or
// soil field (stage 2) or an imposed side (both stages).
struct Variant {
    bool fields;
    int order;  // 1 or 2
    int flux;   // 0 HLL, 1 Rusanov, 2 kinetic
};

using BatchKernel = void (*)(const MemberArgs*, const int4*, int, int, int, double);

template <int STAGE, int TXT, bool FIELDS, int ORDER>
BatchKernel pick_flux(int flux) {
    if constexpr (STAGE == 2 && ORDER == 1) {
        return batch_euler_kernel<TXT, FIELDS>;
    } else {
        switch (flux) {
            case 1: return batch_stage_kernel<STAGE, TXT, FIELDS, ORDER, 1>;
            case 2: return batch_stage_kernel<STAGE, TXT, FIELDS, ORDER, 2>;
            default: return batch_stage_kernel<STAGE, TXT, FIELDS, ORDER, 0>;
        }
    }
}

template <int STAGE, int TXT>
BatchKernel pick_t(const Variant& v) {
    if (v.fields)
        return v.order == 1 ? pick_flux<STAGE, TXT, true, 1>(v.flux)
                            : pick_flux<STAGE, TXT, true, 2>(v.flux);
    return v.order == 1 ? pick_flux<STAGE, TXT, false, 1>(v.flux)
                        : pick_flux<STAGE, TXT, false, 2>(v.flux);
}

template <int STAGE>
BatchKernel pick(int tx, const Variant& v) {
    return tx == 64 ? pick_t<STAGE, 64>(v) : tx == 128 ? pick_t<STAGE, 128>(v)
                                                       : pick_t<STAGE, 256>(v);
}

template <int STAGE>
void launch_batch(const Variant& v, int tx, int grid, hipStream_t s, const MemberArgs* ms,
                  const int4* tiles, int ntiles, int phase, int slot, double t_end) {
    hipLaunchKernelGGL(pick<STAGE>(tx, v), dim3(grid), dim3(tx), 0, s, ms, tiles, ntiles, phase,
                       slot, t_end);
}

}  // namespace

struct swe_batch {
    int count;
    std::vector<swe_params> prm;
    std::vector<MemberArgs> mh;   // host copies of the member table
    std::vector<Backup> bh;       // host copies of the backup table
    MemberArgs* md;               // device member table
    Backup* bd;                   // device backup table
    int4* tiles;                  // device work list
    size_t tiles_cap;
    int ntiles;
    int tx, ty;
    hipStream_t stream;
    int slot;
    size_t max_cells;
    bool any_fields;              // some member has a rain or soil field
    bool any_imposed;             // some member has an imposed side
    int order, flux;              // the members' scheme (shared)
    hipGraphExec_t graph;
    hipStream_t cap_stream;  // private stream used only to capture graphs
    int graph_slot;
    double graph_t_end;
    unsigned graph_epoch;
    unsigned epoch;
};

namespace {

size_t tiles_for(const swe_batch* b, int tx, int ty) {
    size_t n = 0;
    for (int k = 0; k < b->count; ++k)
        n += (size_t)strips_of(b->prm[k].nx, tx) * ((b->prm[k].ny + ty - 1) / ty);
    return n;
}

size_t max_tiles(const swe_params* p, int count) {
    size_t n = 0;
    for (int k = 0; k < count; ++k)
        n += (size_t)strips_of(p[k].nx, 64) * ((p[k].ny + MIN_TY - 1) / MIN_TY);
    return n;
}

int upload_members(swe_batch* b) {
    if (hipMemcpyAsync(b->md, b->mh.data(), sizeof(MemberArgs) * b->count,
                       hipMemcpyHostToDevice, b->stream) != hipSuccess)
        return SWE_EHIP;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return SWE_EHIP;
    b->epoch++;
    return SWE_OK;
}

Variant variant(const swe_batch* b, int stage) {
    return Variant{stage == 1 ? b->any_imposed : (b->any_fields || b->any_imposed), b->order,
                   b->flux};
}

// Work list for a tile shape: members from largest to smallest, each
// member's tiles in strip-major order.
int build_tiles(swe_batch* b, int tx, int ty) {
    size_t n = tiles_for(b, tx, ty);
    if (n > b->tiles_cap || n > (size_t)0x7fffffff) return SWE_EINVAL;
    std::vector<int> order(b->count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        return (size_t)b->prm[a].nx * b->prm[a].ny > (size_t)b->prm[c].nx * b->prm[c].ny;
    });
    std::vector<int4> t;
    t.reserve(n);
    for (int k : order) {
        int strips = strips_of(b->prm[k].nx, tx);
        for (int s = 0; s < strips; ++s)
            for (int y = 0; y < b->prm[k].ny; y += ty)
                t.push_back(make_int4(k, s, y, std::min(y + ty, b->prm[k].ny)));
    }
    if (hipMemcpyAsync(b->tiles, t.data(), sizeof(int4) * t.size(), hipMemcpyHostToDevice,
                       b->stream) != hipSuccess)
        return SWE_EHIP;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return SWE_EHIP;
    b->ntiles = (int)t.size();
    b->tx = tx;
    b->ty = ty;
    b->epoch++;
    return SWE_OK;
}

void enqueue_step(swe_batch* b, int phase, double t_end) {
    launch_batch<1>(variant(b, 1), b->tx, b->ntiles, b->stream, b->md, b->tiles, b->ntiles,
                    phase, b->slot, t_end);
    launch_batch<2>(variant(b, 2), b->tx, b->ntiles, b->stream, b->md, b->tiles, b->ntiles,
                    phase, b->slot, t_end);
    b->slot ^= 1;
}

void drop_graph(swe_batch* b) {
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
}

int ensure_graph(swe_batch* b, double t_end) {
    if (b->graph && b->graph_slot == b->slot && b->graph_t_end == t_end &&
        b->graph_epoch == b->epoch)
        return SWE_OK;
    drop_graph(b);
    int slot0 = b->slot;
    // the caller's stream may be the legacy default stream, which cannot be
    // captured: record on a private stream, launch on the caller's
    if (!b->cap_stream &&
        hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        b->cap_stream = nullptr;
        return SWE_EHIP;
    }
    hipStream_t user = b->stream;
    b->stream = b->cap_stream;
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        b->stream = user;
        return SWE_EHIP;
    }
    for (int k = 0; k < GRAPH_STEPS; ++k) enqueue_step(b, k & 1, t_end);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    b->stream = user;
    b->slot = slot0;
    if (e != hipSuccess || !g) return SWE_EHIP;
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->graph = nullptr;
        return SWE_EHIP;
    }
    b->graph_slot = slot0;
    b->graph_t_end = t_end;
    b->graph_epoch = b->epoch;
    return SWE_OK;
}

int run_steps(swe_batch* b, int32_t nsteps, double t_end, bool use_graph) {
    int32_t k = 0;
    if (use_graph && nsteps >= GRAPH_STEPS) {
        int rc = ensure_graph(b, t_end);
        if (rc) return rc;
        for (; k + GRAPH_STEPS <= nsteps; k += GRAPH_STEPS)
            if (hipGraphLaunch(b->graph, b->stream) != hipSuccess) return SWE_EHIP;
    }
    int phase = 0;
    for (; k < nsteps; ++k) {
        enqueue_step(b, phase, t_end);
        phase ^= 1;
    }
    if (phase == 1)
        hipLaunchKernelGGL(batch_copyback_kernel, dim3(256, b->count), dim3(256), 0, b->stream,
                           (const MemberArgs*)b->md);
    return hip_ok(hipGetLastError());
}

size_t member_bytes(const swe_params& p) {
    size_t an = align256(ncells(&p) * sizeof(double));
    // scalars, second state, rate, backup of the state (+ V_inf), backup scalars
    return SCALAR_BYTES + 3 * an + 3 * an + 3 * an + (p.infil_on ? an : 0) + SCALAR_BYTES;
}

}  // namespace

extern "C" {

int swe_batch_workspace_bytes(const swe_params* p, int32_t count, size_t* bytes) {
    if (!p || count < 1 || !bytes) return SWE_EINVAL;
    size_t total = align256(sizeof(MemberArgs) * count) + align256(sizeof(Backup) * count) +
                   align256(sizeof(int4) * max_tiles(p, count));
    for (int k = 0; k < count; ++k) {
        int rc = check_params(&p[k]);
        if (rc) return rc;
        total += member_bytes(p[k]);
    }
    *bytes = total;
    return SWE_OK;
}

int swe_batch_create(const swe_params* p, const swe_buffers* bufs, int32_t count,
                     void* workspace, size_t workspace_bytes, void* stream, swe_batch** out) {
    size_t need = 0;
    int rc = swe_batch_workspace_bytes(p, count, &need);
    if (rc) return rc;
    if (!bufs || !out || !workspace || ((uintptr_t)workspace & 255) != 0) return SWE_EINVAL;
    if (workspace_bytes < need) return SWE_ENOMEM;
    for (int k = 0; k < count; ++k) {
        const swe_buffers& b = bufs[k];
        if (!b.h || !b.qx || !b.qy || !b.z) return SWE_EINVAL;
        // the members share the scheme (order and flux): one kernel per stage
        if ((p[k].order == 1) != (p[0].order == 1) || p[k].flux != p[0].flux)
            return SWE_EINVAL;
        // the ensemble kernels take MUSCL and the HLL, Rusanov and kinetic
        // fluxes (VFRoe-ncv and the ENO reconstructions: single contexts)
        if (p[k].flux == 3 || (p[k].order != 1 && p[k].recon != 0)) return SWE_EINVAL;
        if (p[k].infil_on && !b.vinf) return SWE_EINVAL;
    }
    swe_batch* b = new (std::nothrow) swe_batch;
    if (!b) return SWE_ENOMEM;
    b->count = count;
    b->prm.assign(p, p + count);
    b->mh.resize(count);
    b->bh.resize(count);
    b->stream = (hipStream_t)stream;
    b->slot = 0;
    b->graph = nullptr;
    b->cap_stream = nullptr;
    b->epoch = 0;
    b->graph_epoch = 0;
    b->max_cells = 0;
    b->any_fields = false;
    b->any_imposed = false;
    b->order = p[0].order == 1 ? 1 : 2;
    b->flux = p[0].flux;
    char* w = (char*)workspace;
    b->md = (MemberArgs*)w;
    w += align256(sizeof(MemberArgs) * count);
    b->bd = (Backup*)w;
    w += align256(sizeof(Backup) * count);
    b->tiles = (int4*)w;
    b->tiles_cap = max_tiles(p, count);
    w += align256(sizeof(int4) * b->tiles_cap);
    for (int k = 0; k < count; ++k) {
        MemberArgs& m = b->mh[k];
        std::memset(&m, 0, sizeof m);
        size_t n = ncells(&p[k]), an = align256(n * sizeof(double));
        b->max_cells = std::max(b->max_cells, n);
        m.p = to_kparams(p[k]);
        m.z = bufs[k].z;
        m.fric = bufs[k].fric;
        m.vinf = p[k].infil_on ? bufs[k].vinf : nullptr;
        attach_fields(m, bufs[k]);
        if (has_fields(m)) b->any_fields = true;
        if (m.p.imposed) b->any_imposed = true;
        m.sc = (DevScalars*)w; w += SCALAR_BYTES;
        m.h[0] = bufs[k].h; m.qx[0] = bufs[k].qx; m.qy[0] = bufs[k].qy;
        m.h[1] = (double*)w; w += an;
        m.qx[1] = (double*)w; w += an;
        m.qy[1] = (double*)w; w += an;
        m.ph = (double*)w; w += an;
        m.pqx = (double*)w; w += an;
        m.pqy = (double*)w; w += an;
        Backup& bk = b->bh[k];
        bk.h = (double*)w; w += an;
        bk.qx = (double*)w; w += an;
        bk.qy = (double*)w; w += an;
        bk.vinf = nullptr;
        if (p[k].infil_on) { bk.vinf = (double*)w; w += an; }
        bk.sc = (DevScalars*)w; w += SCALAR_BYTES;
        hipLaunchKernelGGL(swe_init_scalars_kernel, dim3(1), dim3(64), 0, b->stream, m.sc, 0.0);
    }
    if (hipMemcpyAsync(b->bd, b->bh.data(), sizeof(Backup) * count, hipMemcpyHostToDevice,
                       b->stream) != hipSuccess) {
        delete b;
        return SWE_EHIP;
    }
    rc = upload_members(b);
    // default tile shape (before any autotuning): the single context's
    // strip width for the largest member (one-wave strips below 8M cells),
    // 32 rows for one-wave strips (where the autotuner lands on mixed
    // ensembles), else half the single context's rows for that member
    int big = 0;
    for (int k = 1; k < count; ++k)
        if (ncells(&p[k]) > ncells(&p[big])) big = k;
    const int tx0 = default_tx(p[big].nx, p[big].ny);
    const int ty0 = tx0 == 64 ? 32 : std::max(MIN_TY, auto_rows(p[big].nx, p[big].ny, tx0) / 2);
    if (!rc) rc = build_tiles(b, tx0, ty0);
    if (rc) {
        delete b;
        return rc;
    }
    *out = b;
    return SWE_OK;
}

int swe_batch_destroy(swe_batch* b) {
    if (!b) return SWE_OK;
    drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return SWE_OK;
}

int swe_batch_set_tiling(swe_batch* b, int32_t tx, int32_t ty) {
    if (!b || !valid_tx(tx) || ty < MIN_TY) return SWE_EINVAL;
    return build_tiles(b, tx, ty);
}

int swe_batch_get_tiling(swe_batch* b, int32_t* tx, int32_t* ty, int32_t* ntiles) {
    if (!b) return SWE_EINVAL;
    if (tx) *tx = b->tx;
    if (ty) *ty = b->ty;
    if (ntiles) *ntiles = b->ntiles;
    return SWE_OK;
}

int swe_batch_autotune(swe_batch* b, int32_t trial_steps, int32_t* tx_out, int32_t* ty_out,
                       double* ms_out) {
    if (!b || trial_steps < 2) return SWE_EINVAL;
    trial_steps += trial_steps & 1;
    const int cand_tx[3] = {64, 128, 256};
    const int cand_ty[4] = {8, 16, 32, 64};
    int slot0 = b->slot;
    // save the state once; every candidate starts from it and it is put
    // back at the end, so tuning leaves no trace in the results
    hipLaunchKernelGGL(batch_backup_kernel, dim3(256, b->count), dim3(256), 0, b->stream,
                       (const MemberArgs*)b->md, (const Backup*)b->bd, 0);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return SWE_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return SWE_EHIP; }
    double best = INFINITY;
    int btx = b->tx, bty = b->ty;
    int rc = SWE_OK;
    for (int i = 0; i < 3 && rc == SWE_OK; ++i) {
        for (int j = 0; j < 4 && rc == SWE_OK; ++j) {
            rc = build_tiles(b, cand_tx[i], cand_ty[j]);
            if (rc) break;
            rc = run_steps(b, 2, INFINITY, false);  // warm the caches and code
            if (rc) break;
            (void)hipEventRecord(e0, b->stream);
            rc = run_steps(b, trial_steps, INFINITY, false);
            (void)hipEventRecord(e1, b->stream);
            if (rc) break;
            if (hipEventSynchronize(e1) != hipSuccess) { rc = SWE_EHIP; break; }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) {
                best = ms;
                btx = cand_tx[i];
                bty = cand_ty[j];
            }
            hipLaunchKernelGGL(batch_backup_kernel, dim3(256, b->count), dim3(256), 0,
                               b->stream, (const MemberArgs*)b->md, (const Backup*)b->bd, 1);
            b->slot = slot0;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == SWE_OK) rc = build_tiles(b, btx, bty);
    hipLaunchKernelGGL(batch_backup_kernel, dim3(256, b->count), dim3(256), 0, b->stream,
                       (const MemberArgs*)b->md, (const Backup*)b->bd, 1);
    b->slot = slot0;
    if (hipStreamSynchronize(b->stream) != hipSuccess && rc == SWE_OK) rc = SWE_EHIP;
    if (tx_out) *tx_out = b->tx;
    if (ty_out) *ty_out = b->ty;
    if (ms_out) *ms_out = best / trial_steps;
    return rc;
}

int swe_batch_set_boundary_values(swe_batch* b, int32_t member, int32_t side, double h_b,
                                  double q_b) {
    if (!b || member < 0 || member >= b->count || side < 0 || side > 3) return SWE_EINVAL;
    const int type = b->prm[member].bc[side];
    if (type < SWE_BC_IMPOSED_H || !imposed_values_ok(type, h_b, q_b)) return SWE_EINVAL;
    b->prm[member].bc_h[side] = h_b;
    b->prm[member].bc_q[side] = q_b;
    b->mh[member].p.bc_h[side] = h_b;
    b->mh[member].p.bc_q[side] = q_b;
    return upload_members(b);
}

int swe_batch_set_rain(swe_batch* b, int32_t member, double rain) {
    if (!b || member < 0 || member >= b->count || !(rain >= 0.0) || !std::isfinite(rain))
        return SWE_EINVAL;
    b->prm[member].rain = rain;
    b->mh[member].p.rain = rain;
    return upload_members(b);
}

int swe_batch_set_hyetograph(swe_batch* b, int32_t member, const double* t_pts,
                             const double* r, int32_t n) {
    if (!b || member < 0 || member >= b->count) return SWE_EINVAL;
    HyetoStage st;
    int rc = stage_hyetograph(t_pts, r, n, st);
    if (rc) return rc;
    return upload_hyetograph(b->mh[member].sc, st, b->stream);
}

int swe_batch_set_dt_log(swe_batch* b, int32_t member, double* dev_log, int64_t capacity) {
    if (!b || member < 0 || member >= b->count || capacity < 0) return SWE_EINVAL;
    b->mh[member].dtlog = dev_log;
    b->mh[member].dtlog_cap = dev_log ? capacity : 0;
    return upload_members(b);
}

int swe_batch_step(swe_batch* b, int32_t nsteps, double t_end) {
    Range range("swe_batch_step");
    if (!b || nsteps < 0 || std::isnan(t_end)) return SWE_EINVAL;
    if (nsteps == 0) return SWE_OK;
    return run_steps(b, nsteps, t_end, true);
}

int swe_batch_get_time(swe_batch* b, int32_t member, double* t, double* last_dt,
                       int64_t* steps) {
    if (!b || member < 0 || member >= b->count) return SWE_EINVAL;
    DevScalars s;
    if (hipMemcpyAsync(&s, b->mh[member].sc, sizeof s, hipMemcpyDeviceToHost, b->stream) !=
        hipSuccess)
        return SWE_EHIP;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return SWE_EHIP;
    if (t) *t = s.t[b->slot];
    if (last_dt) *last_dt = s.last_dt;
    if (steps) *steps = s.steps[b->slot];
    return SWE_OK;
}

int swe_batch_get_status(swe_batch* b, uint32_t* flags, int32_t n) {
    if (!b || !flags || n < b->count) return SWE_EINVAL;
    uint32_t any = 0;
    for (int k = 0; k < b->count; ++k) {
        DevScalars s;
        if (hipMemcpyAsync(&s, b->mh[k].sc, sizeof s, hipMemcpyDeviceToHost, b->stream) !=
            hipSuccess)
            return SWE_EHIP;
        if (hipStreamSynchronize(b->stream) != hipSuccess) return SWE_EHIP;
        flags[k] = s.status;
        any |= s.status;
    }
    if (any & SWE_FLAG_NONFINITE) return SWE_ENONFINITE;
    if (any & SWE_FLAG_NEGDEPTH) return SWE_ENEGDEPTH;
    if (any & SWE_FLAG_DT) return SWE_EDT;
    if (any & SWE_FLAG_DT_UNDERFLOW) return SWE_EDTMIN;
    return SWE_OK;
}

}  // extern "C"
