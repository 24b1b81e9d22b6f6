// Eight-neighbour flow directions on a DEM (Section 5.2).
//
// Streaming stencil, bound by HBM: each cell is read once from HBM
// (4 or 8 bytes) and its code written once (1 byte).  A workgroup of 256
// lanes owns a strip of 1024 columns (4 cells per lane) and marches down
// `rows` grid rows, keeping its columns (plus one column on each side) of
// the rows around the current one in registers: every row is loaded once
// per strip, in batches of two rows whose loads are in flight together, and
// the two halo rows of a segment are the only re-reads.  A lane's four
// cells start at a column that is a multiple of 4, so the alignment of
// their address depends on the row only (the same for every lane of the
// row): each row is loaded with the widest loads its alignment allows
// (16, 8 or 4 bytes) and its codes stored as whole 32-, 16- or 8-bit words,
// so rows whose length is not a multiple of 4 keep the wide path.  The last
// lane of a row may hold fewer than four cells.  Codes are written with
// non-temporal stores (they are not read again by the kernel).
//
// Cells outside the grid read as elevation 0, which the strictly-positive
// test never selects, so the boundary needs no special case.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "swe_flowdir.h"

namespace {

constexpr int FD_THREADS = 256;
// rows loaded together per lane: two keeps the kernel within 64 VGPRs (8
// waves per SIMD), which measured faster than four or eight rows in flight
// per lane at 7 or 5 waves, and than one row with no overlap at all
constexpr int FD_BATCH = 2;

template <typename T>
struct Row {
    T v[6];  // columns col0-1 .. col0+4
};

// The four cells col0 .. col0+3 of a row (all inside the grid) with the
// widest loads the address allows; `al` is its alignment in elements
// (4, 2 or 1; the same for the whole row).
__device__ __forceinline__ void load4(const float* p, int al, float* out) {
    if (al == 4) {
        const float4 a = *reinterpret_cast<const float4*>(p);
        out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = a.w;
    } else if (al == 2) {
        const float2 a = reinterpret_cast<const float2*>(p)[0];
        const float2 b = reinterpret_cast<const float2*>(p)[1];
        out[0] = a.x; out[1] = a.y; out[2] = b.x; out[3] = b.y;
    } else {
        out[0] = p[0]; out[1] = p[1]; out[2] = p[2]; out[3] = p[3];
    }
}

__device__ __forceinline__ void load4(const double* p, int al, double* out) {
    if (al >= 2) {
        const double2 a = reinterpret_cast<const double2*>(p)[0];
        const double2 b = reinterpret_cast<const double2*>(p)[1];
        out[0] = a.x; out[1] = a.y; out[2] = b.x; out[3] = b.y;
    } else {
        out[0] = p[0]; out[1] = p[1]; out[2] = p[2]; out[3] = p[3];
    }
}

// Alignment in elements (4, 2 or 1) that the offset e contributes: a power
// of two dividing e, at most 4.  An element's address is aligned to at least
// the smaller of this and the base pointer's alignment (both powers of two).
__device__ __forceinline__ int elem_align(long long e) {
    return (e & 3) == 0 ? 4 : (e & 1) == 0 ? 2 : 1;
}

// Row r of the strip's columns; zeros outside the grid.  `zal` is the
// alignment (in elements) of z itself.
template <typename T>
__device__ __forceinline__ void load_row(const T* __restrict__ z, int nx, int ny, int r,
                                         int col0, int zal, bool active, Row<T>& w) {
#pragma unroll
    for (int k = 0; k < 6; ++k) w.v[k] = T(0);
    if (!active || r < 0 || r >= ny) return;
    const T* row = z + (size_t)r * (size_t)nx;
    if (col0 + 4 <= nx) {
        const int al = min(zal, elem_align((long long)r * nx + col0));
        load4(row + col0, al, &w.v[1]);
    } else {
        for (int k = 0; k < 4; ++k)
            if (col0 + k < nx) w.v[1 + k] = row[col0 + k];
    }
    w.v[0] = col0 > 0 ? row[col0 - 1] : T(0);
    w.v[5] = col0 + 4 < nx ? row[col0 + 4] : T(0);
}

// One step of the scan: keep neighbour v (code k) if it is strictly
// positive and strictly below the running minimum.
template <typename T>
__device__ __forceinline__ void consider(T v, uint32_t k, T& best, uint32_t& code) {
    const bool take = (v > T(0)) & (v < best);
    best = take ? v : best;
    code = take ? k : code;
}

// Code of the cell at window column c (1..4) of the middle row.
template <typename T>
__device__ __forceinline__ uint32_t cell_code(const Row<T>& lo, const Row<T>& mid,
                                              const Row<T>& hi, int c) {
    T best = mid.v[c];
    uint32_t code = 0;
    consider(hi.v[c + 1], 1u, best, code);   // (+1, +1)
    consider(hi.v[c], 2u, best, code);       // (+1,  0)
    consider(hi.v[c - 1], 3u, best, code);   // (+1, -1)
    consider(mid.v[c - 1], 4u, best, code);  // ( 0, -1)
    consider(lo.v[c - 1], 5u, best, code);   // (-1, -1)
    consider(lo.v[c], 6u, best, code);       // (-1,  0)
    consider(lo.v[c + 1], 7u, best, code);   // (-1, +1)
    consider(mid.v[c + 1], 8u, best, code);  // ( 0, +1)
    return code;
}

// The four codes of a lane (packed little-endian) to out, with the widest
// stores its alignment allows; only the first `n` when the row ends sooner.
__device__ __forceinline__ void store_codes(uint8_t* out, uint32_t packed, int al, int n) {
    if (n == 4 && al == 4) {
        __builtin_nontemporal_store(packed, reinterpret_cast<uint32_t*>(out));
    } else if (n == 4 && al == 2) {
        __builtin_nontemporal_store((uint16_t)(packed & 0xffffu), reinterpret_cast<uint16_t*>(out));
        __builtin_nontemporal_store((uint16_t)(packed >> 16), reinterpret_cast<uint16_t*>(out) + 1);
    } else {
        for (int c = 0; c < n; ++c)
            __builtin_nontemporal_store((uint8_t)(packed >> (8 * c)), out + c);
    }
}

template <typename T>
__global__ __launch_bounds__(FD_THREADS) void flow_dir_kernel(const T* __restrict__ z,
                                                              uint8_t* __restrict__ code,
                                                              int nx, int ny, int rows,
                                                              int strips, int zal, int cal) {
    const int b = blockIdx.x;
    const int strip = b % strips;
    const int seg = b / strips;
    const int col0 = (strip * FD_THREADS + (int)threadIdx.x) * 4;
    const bool active = col0 < nx;
    const int ncell = min(4, nx - col0);
    const int y0 = seg * rows;
    const int y1 = min(ny, y0 + rows);

    // w[0], w[1]: rows j0-1 and j0; each batch loads the FD_BATCH rows
    // below them (all loads in flight together), then emits FD_BATCH rows
    Row<T> w[FD_BATCH + 2];
    load_row<T>(z, nx, ny, y0 - 1, col0, zal, active, w[0]);
    load_row<T>(z, nx, ny, y0, col0, zal, active, w[1]);
    for (int j0 = y0; j0 < y1; j0 += FD_BATCH) {
#pragma unroll
        for (int u = 0; u < FD_BATCH; ++u)
            load_row<T>(z, nx, ny, j0 + 1 + u, col0, zal, active && j0 + u < y1, w[2 + u]);
#pragma unroll
        for (int u = 0; u < FD_BATCH; ++u) {
            const int j = j0 + u;
            if (active && j < y1) {
                const long long e = (long long)j * nx + col0;
                uint32_t packed = 0;
#pragma unroll
                for (int c = 1; c <= 4; ++c)
                    packed |= cell_code<T>(w[u], w[u + 1], w[u + 2], c) << (8 * (c - 1));
                store_codes(code + e, packed, min(cal, elem_align(e)), ncell);
            }
        }
        w[0] = w[FD_BATCH];
        w[1] = w[FD_BATCH + 1];
    }
}

// About 4096 workgroups of 1024 columns for float32 and 16384 for float64
// (measured optimum on 8192 x 8192: 16 and 4 rows).
int default_rows(long long nx, long long ny, int elem_bytes) {
    const int shift = elem_bytes == 8 ? 24 : 22;
    long long cells = nx * ny;
    long long r = (cells + (1LL << shift) - 1) >> shift;
    if (r < 4) r = 4;
    if (r > 64) r = 64;
    return (int)r;
}

// Workgroups of flow_dir_kernel<T> the current device holds at once (compute
// units x resident workgroups per unit), or 0 when that cannot be queried.
template <typename T>
int resident_blocks() {
    int dev = -1, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, flow_dir_kernel<T>, FD_THREADS, 0) !=
        hipSuccess)
        return 0;
    return cus * per;
}

// The default rows per workgroup adjusted to the device: a launch runs in
// rounds of `resident` workgroups, each taking about rows + 2 row loads, so
// a last round that is nearly empty costs almost a full one.  Among rows
// within a factor 2 of the default, take the one with the fewest
// rounds x (rows + 2) when that saves more than 15%.
int balanced_rows(long long nx, long long ny, int r0, int resident) {
    if (resident <= 0) return r0;
    const long long strips = (nx + FD_THREADS * 4 - 1) / (FD_THREADS * 4);
    auto cost = [&](long long r) {
        const long long blocks = strips * ((ny + r - 1) / r);
        return ((blocks + resident - 1) / resident) * (r + 2);
    };
    long long best = r0, cbest = cost(r0);
    const long long lo = r0 / 2 < 4 ? 4 : r0 / 2, hi = 2 * r0 > 64 ? 64 : 2 * r0;
    for (long long r = lo; r <= hi; ++r)
        if (cost(r) < cbest) {
            cbest = cost(r);
            best = r;
        }
    return 100 * cbest < 85 * cost(r0) ? (int)best : r0;
}

bool check_args(const void* z, int32_t nx, int32_t ny, const void* code, int32_t rows) {
    if (nx < 0 || ny < 0 || nx > (1 << 30) || rows < 0 || rows > 65536) return false;
    if ((long long)nx * (long long)ny > (1LL << 36)) return false;
    if ((long long)nx * (long long)ny > 0 && (!z || !code)) return false;
    return true;
}

// Alignment in elements of a pointer to `bytes`-byte elements: the largest
// of 4, 2, 1 elements, spanning at most 16 bytes, that divides the address.
int ptr_align(const void* p, int bytes) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    for (int k = 4; k > 1; k /= 2)
        if ((uintptr_t)k * bytes <= 16 && a % ((uintptr_t)k * bytes) == 0) return k;
    return 1;
}

template <typename T>
int flow_dir_launch(const T* z, int32_t nx, int32_t ny, uint8_t* code, int32_t rows,
                    void* stream) {
    if (!check_args(z, nx, ny, code, rows)) return SWE_EINVAL;
    if (nx == 0 || ny == 0) return SWE_OK;
    // alignments of the buffers themselves, in elements; a row's own
    // alignment is the smaller of this and that of its offset
    const int zal = ptr_align(z, (int)sizeof(T));
    const int cal = ptr_align(code, 1);
    const int width = FD_THREADS * 4;
    const long long strips = (nx + width - 1) / width;
    long long r = rows > 0 ? rows
                           : balanced_rows(nx, ny, default_rows(nx, ny, (int)sizeof(T)),
                                           resident_blocks<T>());
    // one-dimensional grid of strips x segments
    while (strips * ((ny + r - 1) / r) > 0x7fffffffLL) r *= 2;
    const long long blocks = strips * ((ny + r - 1) / r);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL((flow_dir_kernel<T>), dim3((unsigned)blocks), dim3(FD_THREADS), 0, s, z,
                       code, (int)nx, (int)ny, (int)r, (int)strips, zal, cal);
    return hipGetLastError() == hipSuccess ? SWE_OK : SWE_EHIP;
}

}  // namespace

extern "C" int swe_flow_dir_f32(const float* z, int32_t nx, int32_t ny, uint8_t* code,
                                int32_t rows, void* hip_stream) {
    return flow_dir_launch<float>(z, nx, ny, code, rows, hip_stream);
}

extern "C" int swe_flow_dir_f64(const double* z, int32_t nx, int32_t ny, uint8_t* code,
                                int32_t rows, void* hip_stream) {
    return flow_dir_launch<double>(z, nx, ny, code, rows, hip_stream);
}

extern "C" int swe_flow_dir_rows(int32_t nx, int32_t ny, int32_t elem_bytes, int32_t* rows) {
    if (!rows || nx < 0 || ny < 0 || (elem_bytes != 4 && elem_bytes != 8)) return SWE_EINVAL;
    const int r0 = default_rows(nx, ny, elem_bytes);
    *rows = balanced_rows(nx, ny, r0,
                          elem_bytes == 4 ? resident_blocks<float>() : resident_blocks<double>());
    return SWE_OK;
}
