"""Pins of the flow-direction oracle (Section 5.2) against what the
definition fixes without running it: closed-form terrains, the tie and
nodata rules, a rotation symmetry, and a brute-force argmin on tiny grids.
Each plausible mistake in the oracle (a wrong comparison, a reordered or
transposed neighbour table, other ghost values) is planted in a copy below
and must fail at least one pin.
"""

import numpy as np
import pytest

from oracle import flowdir as F

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def cone(n, c, sign=1.0, base=1.0, dtype=np.float32):
    r = np.arange(n)[:, None] - c
    s = np.arange(n)[None, :] - c
    return (base + sign * np.sqrt(r * r + s * s)).astype(dtype)


def pin_flat(fd):
    for dtype in (np.float32, np.float64):
        assert not fd(np.full((7, 5), 3.5, dtype)).any()
        assert fd(np.full((1, 1), 2.0, dtype))[0, 0] == 0


def pin_pit(fd):
    # a conical pit: each axis and diagonal cell points one step towards the
    # centre, which gives every code its offset (rows grow with y)
    n, c = 21, 10
    code = fd(cone(n, c))
    assert code[c, c] == 0
    for d in (1, 4, 10):
        assert code[c + d, c] == 6      # above the pit: towards (-1, 0)
        assert code[c - d, c] == 2      # below: (+1, 0)
        assert code[c, c + d] == 4      # east: (0, -1)
        assert code[c, c - d] == 8      # west: (0, +1)
        assert code[c + d, c + d] == 5  # (-1, -1)
        assert code[c + d, c - d] == 7  # (-1, +1)
        assert code[c - d, c + d] == 3  # (+1, -1)
        assert code[c - d, c - d] == 1  # (+1, +1)


def pin_peak_ties(fd):
    # a conical peak: a cell east of the top on the axis has two equally low
    # neighbours, (+1, +1) and (-1, +1); the first in the order (code 1) wins
    n, c = 21, 10
    code = fd(cone(n, c, sign=-1.0, base=100.0))
    for d in (1, 3, 8):
        assert code[c, c + d] == 1
        assert code[c, c - d] == 3      # west: (+1, -1) before (-1, -1)
        assert code[c + d, c] == 1      # above: (+1, +1) before (+1, -1)
        assert code[c - d, c] == 5      # below: (-1, -1) before (-1, +1)


def pin_ramp_and_edges(fd):
    # z rises with x: the three west neighbours tie; the first present in the
    # order is (+1, -1) = 3, or (0, -1) = 4 on the top row; column 0 has no
    # lower neighbour inside the grid and never points at a ghost cell
    ny, nx = 6, 9
    z = (1.0 + np.arange(nx)[None, :] + np.zeros((ny, 1))).astype(np.float32)
    code = fd(z)
    assert (code[:, 0] == 0).all()
    assert (code[:ny - 1, 1:] == 3).all()
    assert (code[ny - 1, 1:] == 4).all()
    # a bowl whose lowest cells are on the border: nothing points outside
    r = np.arange(11)[:, None] - 5.0
    s = np.arange(11)[None, :] - 5.0
    bowl = (50.0 - np.maximum(np.abs(r), np.abs(s))).astype(np.float64)
    cb = fd(bowl)
    jj, ii = np.nonzero(cb)
    for j, i in zip(jj, ii):
        dr, dc = F.OFFSETS[cb[j, i] - 1]
        assert 0 <= j + dr < 11 and 0 <= i + dc < 11


def pin_nodata(fd):
    rng = np.random.default_rng(7)
    z = rng.uniform(1.0, 2.0, (12, 13)).astype(np.float32)
    z[3:6, 4:8] = 0.0
    z[8, 2] = -5.0
    z[0, 12] = -0.0
    code = fd(z)
    ny, nx = z.shape
    for j in range(ny):
        for i in range(nx):
            k = code[j, i]
            if z[j, i] <= 0:
                assert k == 0            # nothing is below a nodata centre
            if k:
                dr, dc = F.OFFSETS[k - 1]
                assert 0 <= j + dr < ny and 0 <= i + dc < nx and z[j + dr, i + dc] > 0
    # a NaN is never selected and a NaN centre keeps code 0
    z[10, 10] = np.nan
    code = fd(z)
    assert code[10, 10] == 0
    for j in range(9, 12):
        for i in range(9, 12):
            k = code[j, i]
            if k:
                dr, dc = F.OFFSETS[k - 1]
                assert (j + dr, i + dc) != (10, 10)


def pin_rotation(fd):
    # rotating the grid a quarter turn (np.rot90) turns offset (dr, dc) into
    # (-dc, dr): code k becomes (k + 5) % 8 + 1 on inputs without ties
    rng = np.random.default_rng(3)
    for shape in ((9, 14), (1, 6), (6, 1)):
        z = rng.permutation(shape[0] * shape[1]).reshape(shape).astype(np.float64) + 1.0
        a = fd(z)
        b = fd(np.ascontiguousarray(np.rot90(z)))
        mapped = np.where(a == 0, 0, (a.astype(int) + 5) % 8 + 1)
        assert np.array_equal(np.rot90(mapped), b)


def brute(z):
    ny, nx = z.shape
    out = np.zeros((ny, nx), np.uint8)
    for j in range(ny):
        for i in range(nx):
            cands = []
            for k, (dr, dc) in enumerate(F.OFFSETS):
                jj, ii = j + dr, i + dc
                if 0 <= jj < ny and 0 <= ii < nx and z[jj, ii] > 0 and z[jj, ii] < z[j, i]:
                    cands.append((z[jj, ii], k))
            if cands:
                out[j, i] = min(cands)[1] + 1
    return out


def pin_brute_force(fd):
    # the lowest admissible neighbour, ties to the smaller code: a
    # lexicographic minimum, not the scan itself
    rng = np.random.default_rng(11)
    for t in range(40):
        ny, nx = int(rng.integers(1, 7)), int(rng.integers(1, 7))
        z = rng.integers(-2, 5, (ny, nx)).astype(np.float32 if t % 2 else np.float64)
        assert np.array_equal(fd(z), brute(z)), z


PINS = [pin_flat, pin_pit, pin_peak_ties, pin_ramp_and_edges, pin_nodata, pin_rotation,
        pin_brute_force]


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_oracle_pinned(pin):
    pin(F.flow_directions)


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_cell_scan_pinned(pin):
    def fd(z):
        ny, nx = z.shape
        return np.array([[F.flow_directions_cell(z, j, i) for i in range(nx)]
                         for j in range(ny)], np.uint8).reshape(ny, nx)
    pin(fd)


# ---------------------------------------------------------------------------
# planted mistakes: each must be caught by some pin
# ---------------------------------------------------------------------------

def scan(z, offsets=F.OFFSETS, lt=np.less, positive=True, ghost=0.0, start_inf=False,
         keep_first=False):
    ny, nx = z.shape
    if isinstance(ghost, str):
        pad = np.pad(z, 1, mode="edge")
    else:
        pad = np.full((ny + 2, nx + 2), ghost, z.dtype)
        pad[1:ny + 1, 1:nx + 1] = z
    best = np.full_like(z, np.inf) if start_inf else z.copy()
    code = np.zeros((ny, nx), np.uint8)
    for k, (dr, dc) in enumerate(offsets):
        nb = pad[1 + dr:1 + dr + ny, 1 + dc:1 + dc + nx]
        take = lt(nb, best)
        if positive:
            take &= nb > 0
        if keep_first:
            take &= code == 0
        code[take] = k + 1
        best = np.where(take, nb, best)
    return code


MUTANTS = {
    "less_equal": lambda z: scan(z, lt=np.less_equal),
    "no_positive_test": lambda z: scan(z, positive=False),
    "reversed_order": lambda z: scan(z, offsets=F.OFFSETS[::-1]),
    "transposed_offsets": lambda z: scan(z, offsets=tuple((c, r) for r, c in F.OFFSETS)),
    "order_rotated_by_one": lambda z: scan(z, offsets=F.OFFSETS[1:] + F.OFFSETS[:1]),
    "ghost_edge_copy": lambda z: scan(z, ghost="edge"),
    "ghost_low": lambda z: scan(z, ghost=0.5, positive=True),
    "start_at_infinity": lambda z: scan(z, start_inf=True),
    "first_lower_not_lowest": lambda z: scan(z, keep_first=True),
    "sign_flip_row": lambda z: scan(z, offsets=tuple((-r, c) for r, c in F.OFFSETS)),
}


def test_unmutated_scan_passes_all_pins():
    for pin in PINS:
        pin(scan)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    fd = MUTANTS[name]
    caught = []
    for pin in PINS:
        try:
            pin(fd)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passes every pin"
