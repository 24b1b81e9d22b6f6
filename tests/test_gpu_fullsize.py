"""Parity at full workload sizes, in the launch configuration bench.py times.

The oracle cannot run thousands of steps on 67M cells, so after the GPU has
advanced the full grid to a representative state, one more GPU step is
checked on sampled cells:
  * the oracle computes the global wave-speed bounds over the whole grid
    and hence dt (which must equal the GPU's dt bit for bit);
  * for each sampled cell, the oracle advances an 11 x 11 window of the
    pre-step state by one step with that dt (a cell's update depends on
    cells at most 4 away, and the window's artificial edges are 5 away) and
    the centre must match the GPU's cell.
Samples include domain corners and edges (where the window uses the true
boundary conditions) and random interior cells.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_1307_4839_amd import inputs as I

pytestmark = pytest.mark.gpu

R = 5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def window_step(wl, st, j, i, dt):
    ny, nx = wl.ny, wl.nx
    j0, j1 = max(0, j - R), min(ny, j + R + 1)
    i0, i1 = max(0, i - R), min(nx, i + R + 1)
    bc = (wl.bc[0] if i0 == 0 else I.OUTFLOW, wl.bc[1] if i1 == nx else I.OUTFLOW,
          wl.bc[2] if j0 == 0 else I.OUTFLOW, wl.bc[3] if j1 == ny else I.OUTFLOW)
    w = I.Workload("win", i1 - i0, j1 - j0, wl.dx, wl.dy,
                   z=np.ascontiguousarray(wl.z[j0:j1, i0:i1]),
                   h=np.ascontiguousarray(st["h"][j0:j1, i0:i1]),
                   qx=np.ascontiguousarray(st["qx"][j0:j1, i0:i1]),
                   qy=np.ascontiguousarray(st["qy"][j0:j1, i0:i1]),
                   bc=bc, g=wl.g, cfl=wl.cfl, dt_max=wl.dt_max, h_eps=wl.h_eps,
                   fric_law=wl.fric_law, fric_coef=wl.fric_coef,
                   fric=None if wl.fric is None else np.ascontiguousarray(wl.fric[j0:j1, i0:i1]),
                   rain=wl.rain, infil_on=wl.infil_on, ks=wl.ks, psi=wl.psi,
                   dtheta=wl.dtheta, order=wl.order, flux=wl.flux, recon=wl.recon,
                   vinf=None if "vinf" not in st else np.ascontiguousarray(st["vinf"][j0:j1, i0:i1]))
    s = oracle.State(w)
    s.step_fixed(dt)
    out = {"h": s.h[j - j0, i - i0], "qx": s.qx[j - j0, i - i0], "qy": s.qy[j - j0, i - i0]}
    if s.vinf is not None:
        out["vinf"] = s.vinf[j - j0, i - i0]
    return out


def sample_cells(nx, ny, n, seed):
    rng = np.random.default_rng(seed)
    pts = [(0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1), (1, nx // 2), (ny - 2, nx // 3),
           (ny // 2, 0), (ny // 2, 1), (ny // 3, nx - 1), (ny // 3, nx - 2)]
    # strip edges of the 252-column tiling and segment edges of 64 rows
    pts += [(ny // 2, 251), (ny // 2, 252), (ny // 2, 253), (63, nx // 2), (64, nx // 2)]
    pts += [(int(rng.integers(0, ny)), int(rng.integers(0, nx))) for _ in range(n)]
    return pts


def check_fullsize(wl, pre_steps, nsamples, seed):
    import torch
    from paper_1307_4839_amd.solver import Solver
    say(f"[fullsize] {wl.name} {wl.nx}x{wl.ny}: {pre_steps} GPU steps")
    g = Solver(wl, dt_log=pre_steps + 2)
    g.step(pre_steps)
    pre = g.state()
    t_pre = g.time()[0]
    g.step(1)
    post = g.state()
    t_post, dt_gpu, steps = g.time()
    rc, flags = g.status()
    assert rc == 0 and flags == 0
    assert np.all(post["h"] >= 0)
    say(f"[fullsize] oracle global bounds over {wl.nx * wl.ny} cells")
    p = oracle.params_of(wl)
    _, _, _, amax = oracle.rate(p, pre["h"], pre["qx"], pre["qy"], wl.z)
    dt = oracle.time_step(p, amax, t_pre, np.inf)
    assert dt == dt_gpu, (dt, dt_gpu)
    assert t_post == t_pre + dt
    say(f"[fullsize] dt = {dt}; checking {nsamples} sampled windows")
    bad = 0
    for (j, i) in sample_cells(wl.nx, wl.ny, nsamples, seed):
        ref = window_step(wl, pre, j, i, dt)
        for k, v in ref.items():
            gv = post[k][j, i]
            scale = max(np.abs(post[k]).max(), 1e-300)
            if abs(gv - v) > 1e-14 * scale:
                bad += 1
                say(f"   mismatch {k} at ({j},{i}): gpu {gv!r} oracle {v!r}")
    assert bad == 0
    del g
    torch.cuda.empty_cache()


def test_fullsize_hillslope_8192():
    wl = I.hillslope_8192()
    check_fullsize(wl, 300, 200, seed=1)


@pytest.mark.parametrize("order,flux,recon", [(1, 0, 0), (2, 1, 0), (2, 2, 0), (2, 3, 0),
                                              (2, 0, 1), (2, 0, 2)])
def test_fullsize_hillslope_8192_scheme_variants(order, flux, recon):
    # the variants bench.py times on the same workload: first order with HLL
    # (n_CFL = 1), the Rusanov, kinetic and VFRoe-ncv fluxes at second order,
    # and the ENO and modified ENO reconstructions
    wl = I.hillslope_8192()
    wl.order, wl.flux, wl.recon = order, flux, recon
    if order == 1:
        wl.cfl = 1.0
    check_fullsize(wl, 300, 100, seed=10 + 3 * order + flux + 7 * recon)


def test_fullsize_valley_2048():
    wl = I.valley_2048()
    check_fullsize(wl, 400, 200, seed=2)


def test_fullsize_calibration_1024():
    wl = I.calibration_1024()
    check_fullsize(wl, 300, 150, seed=3)


def test_fullsize_valley_5120():
    wl = I.valley_5120()
    check_fullsize(wl, 2000, 200, seed=4)


def test_longest_rows():
    # Rows of SWE_MAX_NX cells: a cell's byte offset within its row reaches
    # 2^31 - 8, the top of the range of the kernels' 32-bit lane offsets.
    # One step from the initial state with dt capped by dt_max, so the
    # oracle needs no pass over all 2^29 cells; windows sampled along the
    # whole row: both ends, strip edges of the tiling, the last strip.
    import torch
    from paper_1307_4839_amd import capi
    from paper_1307_4839_amd.solver import Solver
    say("[fullsize] longest rows: generating 2^28 x 2 inputs")
    wl = I.longest_rows()
    nx, ny = wl.nx, wl.ny
    assert nx == capi.SWE_MAX_NX
    g = Solver(wl)
    tx = g.tiling()[0]
    say(f"[fullsize] longest rows: one GPU step, {tx}-column strips")
    g.step(1)
    t, dt_gpu, steps = g.time()
    rc, flags = g.status()
    assert rc == 0 and flags == 0 and steps == 1
    assert dt_gpu == wl.dt_max
    outw = tx - 4
    last = (nx - 1) // outw * outw  # first column of the last strip
    rng = np.random.default_rng(11)
    cols = [0, 1, 2, outw - 1, outw, 4095, 4096, 8191, 8192, nx // 2, last - 1, last, last + 1,
            nx - 4097, nx - 4096, nx - 3, nx - 2, nx - 1]
    cols += [int(c) for c in rng.integers(0, nx, 40)]
    cols += [int(c) for c in rng.integers(nx - (1 << 20), nx, 20)]
    pre = {"h": wl.h, "qx": wl.qx, "qy": wl.qy}
    say(f"[fullsize] longest rows: {ny * len(cols)} sampled windows")
    refs, gpus = [], []
    for j in range(ny):
        for i in cols:
            refs.append(window_step(wl, pre, j, i, wl.dt_max))
            gpus.append({k: getattr(g, k)[j, i].item() for k in ("h", "qx", "qy")})
    bad = 0
    for k in ("h", "qx", "qy"):
        scale = max(max(abs(r[k]) for r in refs), 1e-300)
        for n, (r, v) in enumerate(zip(refs, gpus)):
            if abs(v[k] - r[k]) > 1e-14 * scale:
                bad += 1
                say(f"   mismatch {k} at sample {n}: gpu {v[k]!r} oracle {r[k]!r}")
    # the sampled cells are not all still: the step moved water
    assert max(abs(r["qx"]) for r in refs) > 0
    assert bad == 0
    del g
    torch.cuda.empty_cache()
