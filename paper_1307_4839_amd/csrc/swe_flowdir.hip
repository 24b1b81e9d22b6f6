// Eight-neighbour flow directions on a DEM (Section 5.2).
//
// Streaming stencil, bound by HBM: each cell is read once from HBM
// (4 or 8 bytes) and its code written once (1 byte).  A workgroup of 256
// lanes owns a strip of 256*V columns (V = 4 cells per lane on aligned
// rows, else 1) and marches down `rows` grid rows, keeping its columns
// (plus one column on each side) of the rows around the current one in
// registers: every row is loaded once per strip, in batches of two rows
// whose loads are in flight together, and the two halo rows of a segment
// are the only re-reads.  Codes are written with non-temporal stores (they
// are not read again by the kernel).
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

template <typename T, int V>
struct Row {
    T v[V + 2];  // columns col0-1 .. col0+V
};

template <typename T>
__device__ __forceinline__ void load_vec4(const T* p, T* out);

template <>
__device__ __forceinline__ void load_vec4<float>(const float* p, float* out) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = a.w;
}

template <>
__device__ __forceinline__ void load_vec4<double>(const double* p, double* out) {
    const double2 a = reinterpret_cast<const double2*>(p)[0];
    const double2 b = reinterpret_cast<const double2*>(p)[1];
    out[0] = a.x; out[1] = a.y; out[2] = b.x; out[3] = b.y;
}

// Row r of the strip's columns; zeros outside the grid.
template <typename T, int V>
__device__ __forceinline__ void load_row(const T* __restrict__ z, int nx, int ny, int r,
                                         int col0, bool active, Row<T, V>& w) {
    if (!active || r < 0 || r >= ny) {
#pragma unroll
        for (int k = 0; k < V + 2; ++k) w.v[k] = T(0);
        return;
    }
    const T* row = z + (size_t)r * (size_t)nx;
    if constexpr (V == 4) {
        load_vec4<T>(row + col0, &w.v[1]);
    } else {
        w.v[1] = row[col0];
    }
    w.v[0] = col0 > 0 ? row[col0 - 1] : T(0);
    w.v[V + 1] = col0 + V < nx ? row[col0 + V] : T(0);
}

// One step of the scan: keep neighbour v (code k) if it is strictly
// positive and strictly below the running minimum.
template <typename T>
__device__ __forceinline__ void consider(T v, uint32_t k, T& best, uint32_t& code) {
    const bool take = (v > T(0)) & (v < best);
    best = take ? v : best;
    code = take ? k : code;
}

// Code of the cell at window column c (1..V) of the middle row.
template <typename T, int V>
__device__ __forceinline__ uint32_t cell_code(const Row<T, V>& lo, const Row<T, V>& mid,
                                              const Row<T, V>& hi, int c) {
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

template <typename T, int V>
__global__ __launch_bounds__(FD_THREADS) void flow_dir_kernel(const T* __restrict__ z,
                                                              uint8_t* __restrict__ code,
                                                              int nx, int ny, int rows,
                                                              int strips) {
    const int b = blockIdx.x;
    const int strip = b % strips;
    const int seg = b / strips;
    const int col0 = (strip * FD_THREADS + (int)threadIdx.x) * V;
    const bool active = col0 < nx;
    const int y0 = seg * rows;
    const int y1 = min(ny, y0 + rows);

    // w[0], w[1]: rows j0-1 and j0; each batch loads the FD_BATCH rows
    // below them (all loads in flight together), then emits FD_BATCH rows
    Row<T, V> w[FD_BATCH + 2];
    load_row<T, V>(z, nx, ny, y0 - 1, col0, active, w[0]);
    load_row<T, V>(z, nx, ny, y0, col0, active, w[1]);
    for (int j0 = y0; j0 < y1; j0 += FD_BATCH) {
#pragma unroll
        for (int u = 0; u < FD_BATCH; ++u)
            load_row<T, V>(z, nx, ny, j0 + 1 + u, col0, active && j0 + u < y1, w[2 + u]);
#pragma unroll
        for (int u = 0; u < FD_BATCH; ++u) {
            const int j = j0 + u;
            if (active && j < y1) {
                uint8_t* out = code + (size_t)j * (size_t)nx + col0;
                if constexpr (V == 4) {
                    uint32_t packed = 0;
#pragma unroll
                    for (int c = 1; c <= 4; ++c)
                        packed |= cell_code<T, V>(w[u], w[u + 1], w[u + 2], c) << (8 * (c - 1));
                    __builtin_nontemporal_store(packed, reinterpret_cast<uint32_t*>(out));
                } else {
                    __builtin_nontemporal_store((uint8_t)cell_code<T, V>(w[u], w[u + 1], w[u + 2], 1),
                                                out);
                }
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

bool check_args(const void* z, int32_t nx, int32_t ny, const void* code, int32_t rows) {
    if (nx < 0 || ny < 0 || nx > (1 << 30) || rows < 0 || rows > 65536) return false;
    if ((long long)nx * (long long)ny > (1LL << 36)) return false;
    if ((long long)nx * (long long)ny > 0 && (!z || !code)) return false;
    return true;
}

template <typename T>
int flow_dir_launch(const T* z, int32_t nx, int32_t ny, uint8_t* code, int32_t rows,
                    void* stream) {
    if (!check_args(z, nx, ny, code, rows)) return SWE_EINVAL;
    if (nx == 0 || ny == 0) return SWE_OK;
    const bool vec = nx % 4 == 0 && reinterpret_cast<uintptr_t>(z) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(code) % 4 == 0;
    const int width = FD_THREADS * (vec ? 4 : 1);
    const long long strips = (nx + width - 1) / width;
    long long r = rows > 0 ? rows : default_rows(nx, ny, (int)sizeof(T));
    // one-dimensional grid of strips x segments
    while (strips * ((ny + r - 1) / r) > 0x7fffffffLL) r *= 2;
    const long long blocks = strips * ((ny + r - 1) / r);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (vec)
        hipLaunchKernelGGL((flow_dir_kernel<T, 4>), dim3((unsigned)blocks), dim3(FD_THREADS), 0,
                           s, z, code, (int)nx, (int)ny, (int)r, (int)strips);
    else
        hipLaunchKernelGGL((flow_dir_kernel<T, 1>), dim3((unsigned)blocks), dim3(FD_THREADS), 0,
                           s, z, code, (int)nx, (int)ny, (int)r, (int)strips);
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
    *rows = default_rows(nx, ny, elem_bytes);
    return SWE_OK;
}
