"""Ensemble (uneven members in one persistent launch per stage), tile-shape
invariance and graph replay, through the C ABI.

Every member must evolve bit for bit as in its own single-simulation
context (which is itself checked against the oracle), for every tile
shape; the autotuner must leave no trace; graph replays must equal eager
stepping at every replay.
"""

import math
import sys

import numpy as np
import pytest

import oracle
from paper_1307_4839_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def members():
    out = []
    for k, n in enumerate([37, 64, 90, 130, 253, 300]):
        wl = I.ensemble_member(k, n=n)
        wl.rain = (1 + k) * 1e-3  # wet quickly
        out.append(wl)
    # heterogeneous physics: a dam break with Manning, a Green-Ampt hillslope,
    # a friction field, a non-square grid
    out.append(I.dam_break_200(77, 51))
    h = I.hillslope_8192(120, 70)
    h.rain = 2e-3
    out.append(h)
    out.append(I.calibration_1024(140, 160, dam_row=30, ngauges=4, sigma_cells=5))
    out.append(I.random_state(45, 260, seed=5, bc=(1, 0, 0, 1), fric_law=2, fric_coef=0.1))
    return out


def run_single(wl, nsteps):
    from paper_1307_4839_amd.solver import Solver
    g = Solver(wl)
    g.step(nsteps)
    st = g.state()
    st["t"] = g.time()[0]
    g.close()
    return st


def same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("h", "qx", "qy")) and \
        (("vinf" not in a) or np.array_equal(a["vinf"], b["vinf"]))


def test_ensemble_members_equal_single_runs(torch_cuda):
    from paper_1307_4839_amd.solver import Ensemble
    wls = members()
    n = 37
    ref = [run_single(wl, n) for wl in wls]
    for tx, ty in [(256, 16), (128, 8), (64, 4), (256, 64)]:
        say(f"[ensemble] tiling {tx}x{ty}")
        e = Ensemble(wls)
        e.set_tiling(tx, ty)
        e.step(n)
        rc, flags = e.status()
        assert rc == 0 and not any(flags)
        for k, wl in enumerate(wls):
            st = e.state(k)
            assert same(st, ref[k]), (tx, ty, k, wl.name)
            assert e.time(k)[0] == ref[k]["t"]
        e.close()


def test_ensemble_member_against_oracle(torch_cuda):
    from paper_1307_4839_amd.solver import Ensemble
    wls = members()
    e = Ensemble(wls)
    e.step(25)
    for k in (0, 6, 7, 8):
        s = oracle.State(wls[k])
        assert s.run(25) == 0
        st = e.state(k)
        for f in ("h", "qx", "qy"):
            ref = getattr(s, f)
            err = np.abs(st[f] - ref).max() / max(np.abs(ref).max(), 1e-300)
            assert err <= 1e-12, (k, f, err)
        assert e.time(k)[0] == s.t


def test_autotune_leaves_no_trace(torch_cuda):
    from paper_1307_4839_amd.solver import Ensemble
    wls = members()
    a = Ensemble(wls)
    a.step(5)
    tx, ty, ms = a.autotune(4)
    say(f"[ensemble] autotune chose {tx}x{ty} ({ms:.3f} ms/step)")
    assert tx in (64, 128, 256) and ty in (8, 16, 32, 64) and ms > 0
    a.step(20)
    b = Ensemble(wls)
    b.step(25)
    for k in range(len(wls)):
        assert same(a.state(k), b.state(k)), k
        assert a.time(k) == b.time(k)


def test_ensemble_graph_replay_equals_eager(torch_cuda):
    from paper_1307_4839_amd.solver import Ensemble
    wls = members()
    g = Ensemble(wls)   # 16-step calls replay the captured graph
    e = Ensemble(wls)   # 4-step calls run eagerly
    for rep in range(3):
        g.step(16)
        for _ in range(4):
            e.step(4)
        for k in range(len(wls)):
            assert same(g.state(k), e.state(k)), (rep, k)


def test_single_tiling_invariance_and_graph_replay(torch_cuda):
    from paper_1307_4839_amd.solver import Solver
    wl = I.hillslope_8192(700, 300)
    wl.rain = 5e-3
    ref = None
    for tx, ty in [(256, 0), (128, 8), (64, 3), (256, 64), (128, 300)]:
        g = Solver(wl)
        g.set_tiling(tx, ty)
        g.step(20)
        st = g.state()
        if ref is None:
            ref = st
        else:
            assert same(st, ref), (tx, ty)
        g.close()
    # graph replays with eager work and synchronizations in between
    a = Solver(wl)
    b = Solver(wl)
    for rep in range(3):
        a.step(16)
        sa = a.state()
        for _ in range(16):
            b.step(1)
        assert same(sa, b.state()), rep
        assert a.time() == b.time()


def test_bench_ensemble_configuration(torch_cuda):
    # the 256-member ensemble bench.py times (autotuned tiling, graph
    # replay): sampled members bit-identical to their own runs and, for the
    # smallest, within 1e-12 of the oracle
    from paper_1307_4839_amd.solver import Ensemble
    wls = I.ensemble(256)
    e = Ensemble(wls)
    e.autotune(4)
    n = 40
    e.step(n)
    rc, flags = e.status()
    assert rc == 0 and not any(flags)
    sizes = [wl.nx * wl.ny for wl in wls]
    picks = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), 0, 17, 128, 255})
    for k in picks:
        ref = run_single(wls[k], n)
        assert same(e.state(k), ref), k
        assert e.time(k)[0] == ref["t"]
    k = int(np.argmin(sizes))
    s = oracle.State(wls[k])
    assert s.run(n) == 0
    st = e.state(k)
    for f in ("h", "qx", "qy"):
        ref = getattr(s, f)
        assert np.abs(st[f] - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-300), f
    e.close()
