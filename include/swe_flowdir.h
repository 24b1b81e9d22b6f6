/*
 * swe_flowdir.h -- C ABI of the eight-neighbour flow-direction kernel of
 * the same library (arXiv:1307.4839, Section 5.2: the flow-direction step
 * of watershed delineation, given there as the example of an
 * eight-neighbour computation on a DEM).
 *
 * For each cell of an elevation grid z the kernel visits the eight
 * neighbours in a fixed order, keeps a running minimum that starts at the
 * cell's own elevation, and replaces it only by a neighbour whose elevation
 * is strictly positive and strictly lower than the current minimum.  The
 * code written for the cell is the 1-based position, in that order, of the
 * neighbour kept last, or 0 when no neighbour qualifies.  Order, as
 * (row offset, column offset) with rows growing with y:
 *     1:(+1,+1)  2:(+1,0)  3:(+1,-1)  4:(0,-1)
 *     5:(-1,-1)  6:(-1,0)  7:(-1,+1)  8:(0,+1)
 * Consequences: ties go to the smaller code; cells outside the grid count
 * as elevation 0 and are never selected, as is any neighbour with
 * elevation <= 0 (nodata) or NaN; a cell whose own elevation is <= 0 or NaN
 * gets code 0.  Only comparisons are made, so the result is exact.
 *
 * Conventions: z is [ny][nx] row-major with x fastest, no padding, in
 * device memory; code is [ny][nx] uint8 in device memory.  Both buffers
 * are owned by the caller and must not overlap.  The call is asynchronous:
 * it enqueues one kernel on hip_stream (NULL = the default stream) and
 * returns.  Any row length is accepted, and any placement of the buffers
 * provided z is aligned to its element size (4 or 8 bytes): each lane
 * reads its four cells of a row with the widest loads their alignment
 * allows (16, 8 or 4 bytes) and stores their codes as one aligned 32-bit
 * word (joined across two lanes when the row's codes do not start on a
 * 4-byte boundary).
 */
#ifndef SWE_FLOWDIR_H
#define SWE_FLOWDIR_H

#include <stdint.h>

#include "swe.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Flow directions of a float32 DEM (the element type of the paper's
 * example).  rows: grid rows per workgroup, 0 for the default (it is raised
 * where needed to keep the launch grid within its limits).
 * Returns SWE_OK (also for nx == 0 or ny == 0, with nothing launched),
 * SWE_EINVAL for nx or ny negative, more than 2^36 cells, rows negative or
 * above 65536, a null pointer with cells to process or a z not aligned to
 * its element size, and SWE_EHIP if the launch fails. */
int swe_flow_dir_f32(const float* z, int32_t nx, int32_t ny, uint8_t* code,
                     int32_t rows, void* hip_stream);

/* The same on a float64 DEM (e.g. the bed elevation of a simulation). */
int swe_flow_dir_f64(const double* z, int32_t nx, int32_t ny, uint8_t* code,
                     int32_t rows, void* hip_stream);

/* Rows per workgroup that swe_flow_dir_f32 (elem_bytes 4) or
 * swe_flow_dir_f64 (elem_bytes 8) uses for rows == 0, before any raise for
 * the grid limit: about 6144 (float) or 16384 (double) workgroups of 1024
 * columns, within [4, 64].  Host only, no device call; SWE_EINVAL for other
 * elem_bytes, negative sizes or a null rows. */
int swe_flow_dir_rows(int32_t nx, int32_t ny, int32_t elem_bytes, int32_t* rows);

#ifdef __cplusplus
}
#endif

#endif /* SWE_FLOWDIR_H */
