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
// (16, 8 or 4 bytes), and its codes are stored as aligned 32-bit words: on a
// row whose codes do not start on a 4-byte boundary, each lane joins its
// last codes with the next lane's first ones (a lane shift), so rows whose
// length is not a multiple of 4 keep whole-word stores.  The last lane of a
// row may hold fewer than four cells.  Codes of rows that start on a cache
// line are written with non-temporal stores (they are not read again by the
// kernel), the others through the cache (see store_codes).
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

// Value of lane t+1 of the wave (lane 63 gets its own), by a full-wave DPP
// shift.
__device__ __forceinline__ uint32_t from_next_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x130, 0xf, 0xf, false);
}

// Bytes [b0, b1) of a lane's packed codes to out + b0, with the widest
// aligned stores that fit (at most three stores).
__device__ __forceinline__ void store_bytes(uint8_t* out, uint32_t packed, int b0, int b1) {
    int b = b0;
    while (b < b1) {
        const uintptr_t a = reinterpret_cast<uintptr_t>(out + b);
        if (b1 - b >= 2 && (a & 1) == 0) {
            *reinterpret_cast<uint16_t*>(out + b) = (uint16_t)(packed >> (8 * b));
            b += 2;
        } else {
            out[b] = (uint8_t)(packed >> (8 * b));
            b += 1;
        }
    }
}

// The `n` codes of a lane (packed little-endian, n = 4 but for the last
// lane of a row) to out.  A row whose codes start on a 4-byte boundary is
// one 32-bit store per lane.  On a row whose codes start s = 1..3 bytes
// before a boundary, every lane stores one aligned 32-bit word made of its
// last 4 - s codes and the first s codes of the next lane (taken by a lane
// shift), and only the wave's first lane, its last lane and the end of the
// row store single bytes or halves.  `line`: the row's codes start on a
// 128-byte cache line, so every wave writes whole lines, and the stores
// are non-temporal (the codes are not read again); other rows store through
// the cache, where the lines that two waves share are merged before they
// are written to memory (non-temporal stores of such rows wrote about 1.19
// times the code bytes, these 1.05).  `lane` is the lane in the wave; all
// lanes of a wave that are left of an active lane are active with n = 4.
__device__ __forceinline__ void store_codes(uint8_t* out, uint32_t packed, int s, int n,
                                            int n_next, int lane, bool line) {
    if (s == 0) {
        if (n < 4) {
            store_bytes(out, packed, 0, n);
        } else if (line) {
            __builtin_nontemporal_store(packed, reinterpret_cast<uint32_t*>(out));
        } else {
            // keeps the compiler from hoisting this store and the
            // non-temporal one above into one store without the hint
            asm volatile("" ::: "memory");
            *reinterpret_cast<uint32_t*>(out) = packed;
        }
        return;
    }
    // the next lane's codes (every lane of the wave takes part in the shift)
    const uint32_t next = from_next_lane(packed);
    // the word at out + s: this lane's codes s..3 and the next lane's 0..s-1
    const bool join = lane < 63 && n == 4 && n_next >= s;
    // codes 0..s-1 go into the previous lane's word unless this lane is the
    // wave's first or the previous lane did not join (this lane then holds
    // fewer than s codes)
    const bool lead = lane == 0 || n < s;
    if (lead) store_bytes(out, packed, 0, min(s, n));
    if (join) {
        *reinterpret_cast<uint32_t*>(out + s) = (packed >> (8 * s)) | (next << (32 - 8 * s));
    } else if (n > s) {
        store_bytes(out, packed, s, n);
    }
}

template <typename T>
__global__ __launch_bounds__(FD_THREADS) void flow_dir_kernel(const T* __restrict__ z,
                                                              uint8_t* __restrict__ code,
                                                              int nx, int ny, int rows,
                                                              int strips, int zal, int cal0) {
    const int b = blockIdx.x;
    const int strip = b % strips;
    const int seg = b / strips;
    const int col0 = (strip * FD_THREADS + (int)threadIdx.x) * 4;
    const bool active = col0 < nx;
    const int ncell = active ? min(4, nx - col0) : 0;
    // codes held by the next lane of the row (0 past its end)
    const int ncell_next = col0 + 4 < nx ? min(4, nx - col0 - 4) : 0;
    const int lane = (int)threadIdx.x & 63;
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
            // rows past the segment's end are the same for every lane: the
            // whole wave skips them, so the lane shift of store_codes sees
            // every lane of the wave
            if (j < y1) {
                const long long e = (long long)j * nx + col0;
                uint32_t packed = 0;
#pragma unroll
                for (int c = 1; c <= 4; ++c)
                    packed |= cell_code<T>(w[u], w[u + 1], w[u + 2], c) << (8 * (c - 1));
                // bytes from the codes' start to the next 4-byte boundary
                // (the same for every lane of the row), and whether the
                // row's codes start on a cache line
                const int s = (int)((4 - ((cal0 + e) & 3)) & 3);
                const bool line = ((cal0 + (long long)j * nx) & 127) == 0;
                store_codes(code + e, packed, s, ncell, ncell_next, lane, line);
            }
        }
        w[0] = w[FD_BATCH];
        w[1] = w[FD_BATCH + 1];
    }
}

// Rows per workgroup: about 6144 workgroups of 1024 columns for float32 and
// 16384 for float64, within [4, 64] (measured on 8192 x 8192, 14786 x 10086
// and nearby widths: 8 to 16 rows and 24 rows for float32, 4 rows for
// float64, are the fastest or within 2% of it).
int default_rows(long long nx, long long ny, int elem_bytes) {
    const long long cells = nx * ny;
    const long long per = elem_bytes == 8 ? (16384LL << 10) : (6144LL << 10);
    long long r = (cells + per / 2) / per;
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
    const uintptr_t za = reinterpret_cast<uintptr_t>(z);
    if (za % sizeof(T) != 0) return SWE_EINVAL;  // z must be aligned to its element
    // z's own alignment in elements (at most 16 bytes; a row's is the
    // smaller of this and that of its offset) and the codes' address mod 128
    const int zal = za % 16 == 0 ? 16 / (int)sizeof(T) : za % 8 == 0 ? 8 / (int)sizeof(T) : 1;
    const int cal0 = (int)(reinterpret_cast<uintptr_t>(code) & 127);
    const int width = FD_THREADS * 4;
    const long long strips = (nx + width - 1) / width;
    long long r = rows > 0 ? rows : default_rows(nx, ny, (int)sizeof(T));
    // one-dimensional grid of strips x segments
    while (strips * ((ny + r - 1) / r) > 0x7fffffffLL) r *= 2;
    const long long blocks = strips * ((ny + r - 1) / r);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL((flow_dir_kernel<T>), dim3((unsigned)blocks), dim3(FD_THREADS), 0, s, z,
                       code, (int)nx, (int)ny, (int)r, (int)strips, zal, cal0);
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
