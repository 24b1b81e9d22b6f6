"""CPU oracle for the eight-neighbour flow-direction computation of
Section 5.2 (test infrastructure only: tests, the smoke check and the
benchmark's CPU-baseline leg may use it; nothing in the library does).

The paper's user function (Section 5.2, the function given to the
skeleton) visits the eight neighbours of a cell in a fixed order, keeps the
running minimum starting from the cell's own elevation, and replaces it only
by a neighbour whose elevation is strictly positive and strictly below the
current minimum; the output is the 1-based position of the last replacement
in that order, 0 if none.  Read this way:

* neighbour order: the eight shifts of the paper's skeleton composition,
  in the order they appear there, read as (row offset, column offset) with
  rows increasing with y:  1:(+1,+1) 2:(+1,0) 3:(+1,-1) 4:(0,-1)
  5:(-1,-1) 6:(-1,0) 7:(-1,+1) 8:(0,+1);
* a neighbour outside the grid is a ghost cell of elevation 0, which the
  "strictly positive" test never selects (the same rule as a nodata cell
  stored as 0 or a negative value);
* strict comparisons, so among equal lowest neighbours the first in the
  order wins; a NaN elevation is never selected (every comparison with it is
  false) and a NaN centre keeps code 0.

Elevations are compared in the input's own precision (float32 in the
paper's listing; float64 also accepted), with no arithmetic at all, so the
result is exact.  Codes are uint8.
"""

from __future__ import annotations

import numpy as np

# (row offset, column offset) of codes 1..8
OFFSETS = ((1, 1), (1, 0), (1, -1), (0, -1), (-1, -1), (-1, 0), (-1, 1), (0, 1))


def flow_directions(z: np.ndarray) -> np.ndarray:
    """Codes 0..8 per cell of the [ny][nx] elevation array ``z``."""
    z = np.asarray(z)
    if z.ndim != 2 or z.dtype not in (np.float32, np.float64):
        raise ValueError("z must be a 2-D float32 or float64 array")
    ny, nx = z.shape
    # one ghost layer of elevation 0 around the grid
    pad = np.zeros((ny + 2, nx + 2), dtype=z.dtype)
    pad[1:ny + 1, 1:nx + 1] = z
    best = z.copy()
    code = np.zeros((ny, nx), dtype=np.uint8)
    # the eight neighbours in order; each visit is the paper's scan step
    # applied to every cell at once
    for k, (dr, dc) in enumerate(OFFSETS):
        nb = pad[1 + dr:1 + dr + ny, 1 + dc:1 + dc + nx]
        take = (nb > 0) & (nb < best)
        code[take] = k + 1
        best = np.where(take, nb, best)
    return code


def flow_directions_cell(z: np.ndarray, j: int, i: int) -> int:
    """The same scan for one cell, with plain Python loops (for sampled
    checks of large grids)."""
    ny, nx = z.shape
    best = z[j, i]
    code = 0
    for k, (dr, dc) in enumerate(OFFSETS):
        jj, ii = j + dr, i + dc
        v = z[jj, ii] if (0 <= jj < ny and 0 <= ii < nx) else z.dtype.type(0)
        if v > 0 and v < best:
            code = k + 1
            best = v
    return code
