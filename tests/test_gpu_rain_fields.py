"""GPU parity of rain R(t, x, y) = r(t) w(x, y) (hyetograph times a per-cell
weight) and per-cell Green-Ampt parameters, through the C ABI: single
contexts against the oracle, ensemble members against their own single
runs, a hyetograph replaced between steps (graph replays read the new
table), and the argument checks of swe_set_hyetograph.
"""

import math
import sys

import numpy as np
import pytest

import oracle
from paper_1307_4839_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def with_fields(wl, seed, rain=True, soil=True):
    rng = np.random.default_rng(seed)
    wl = wl.copy()
    if rain:
        # breakpoints on whole seconds: the dry start steps by dt_max = 1 s,
        # so several of them are exactly a step's start time
        wl.rain_t = np.array([0.0, 60.0, 150.0, 220.0, 300.0])
        wl.rain_r = np.array([50.0, 120.0, 0.0, 80.0, 30.0]) * I.MM_PER_HOUR
        wl.rain_w = 0.2 + 1.6 * (0.5 + 0.5 * I.smooth_field(rng, wl.nx, wl.ny, 8.0))
    if soil and wl.infil_on:
        shape = (wl.ny, wl.nx)
        wl.ks_f = wl.ks * rng.uniform(0.5, 1.5, shape)
        wl.psi_f = wl.psi * rng.uniform(0.5, 1.5, shape)
        wl.dtheta_f = wl.dtheta * rng.uniform(0.7, 1.3, shape)
    return wl


def compare(wl, nsteps):
    from paper_1307_4839_amd.solver import Solver
    say(f"[rain] {wl.name} {wl.nx}x{wl.ny} steps={nsteps} hyetograph={wl.rain_t is not None} "
        f"weight={wl.rain_w is not None} soil={wl.ks_f is not None}")
    s = oracle.State(wl)
    assert s.run(nsteps) == 0
    g = Solver(wl, dt_log=nsteps)
    g.step(nsteps)
    rc, flags = g.status()
    assert rc == 0 and flags == 0
    t, _, steps = g.time()
    assert steps == s.steps and t == s.t
    assert np.array_equal(g.dts(), np.array(s.dts))
    st = g.state()
    for k in ("h", "qx", "qy", "vinf"):
        if k in st:
            e = rel_err(st[k], getattr(s, k))
            say(f"    {k}: rel err {e:.3e} bitwise={np.array_equal(st[k], getattr(s, k))}")
            assert e <= TOL, k
    g.close()
    return s, st


def test_hyetograph_weight_and_soil_fields(torch_cuda):
    wl = with_fields(I.hillslope_8192(300, 260), seed=1)
    s, st = compare(wl, 650)
    assert s.t > 300.0 and (s.h > 0).any()  # every breakpoint crossed


def test_hyetograph_only_constant_soil(torch_cuda):
    wl = with_fields(I.hillslope_8192(253, 130), seed=2, soil=False)
    wl.rain_w = None
    compare(wl, 350)


def test_soil_fields_only(torch_cuda):
    wl = with_fields(I.hillslope_8192(131, 257), seed=3, rain=False)
    compare(wl, 300)


def test_one_wave_strips(torch_cuda):
    # the same physics on 64-column strips (DPP neighbour exchange)
    from paper_1307_4839_amd.solver import Solver
    wl = with_fields(I.hillslope_8192(300, 140), seed=4)
    s = oracle.State(wl)
    assert s.run(300) == 0
    g = Solver(wl)
    g.set_tiling(64, 8)
    g.step(300)
    st = g.state()
    for k in ("h", "qx", "qy", "vinf"):
        assert rel_err(st[k], getattr(s, k)) <= TOL, k
    g.close()


def test_fields_equal_to_scalars_are_bit_identical(torch_cuda):
    from paper_1307_4839_amd.solver import Solver
    base = I.hillslope_8192(200, 120)
    wl = base.copy()
    shape = (wl.ny, wl.nx)
    wl.rain_w = np.ones(shape)
    wl.ks_f = np.full(shape, wl.ks)
    wl.psi_f = np.full(shape, wl.psi)
    wl.dtheta_f = np.full(shape, wl.dtheta)
    a, b = Solver(base), Solver(wl)
    a.step(300)
    b.step(300)
    sa, sb = a.state(), b.state()
    for k in ("h", "qx", "qy", "vinf"):
        assert np.array_equal(sa[k], sb[k]), k
    a.close()
    b.close()


def test_hyetograph_replaced_between_steps(torch_cuda):
    # 40 steps on one table, then a new one: the graph-replayed steps after
    # the change must read it (the table lives in device memory)
    from paper_1307_4839_amd.solver import Solver
    wl = with_fields(I.hillslope_8192(160, 150), seed=5)
    wl2 = wl.copy()
    wl2.rain_t = np.array([0.0, 45.0, 90.0])
    wl2.rain_r = np.array([10.0, 200.0, 5.0]) * I.MM_PER_HOUR
    s = oracle.State(wl)
    assert s.run(40) == 0
    s.p = oracle.params_of(wl2)
    assert s.run(100) == 0
    g = Solver(wl)
    g.step(40)
    g.set_hyetograph(wl2.rain_t, wl2.rain_r)
    g.step(100)
    st = g.state()
    for k in ("h", "qx", "qy", "vinf"):
        assert rel_err(st[k], getattr(s, k)) <= TOL, k
    # removing the table falls back to the constant rain of the parameters
    # (the weight and soil fields stay)
    wl3 = wl.copy()
    wl3.rain_t = wl3.rain_r = None
    s.p = oracle.params_of(wl3)
    assert s.run(30) == 0
    g.set_hyetograph(None, None)
    g.step(30)
    st = g.state()
    for k in ("h", "qx", "qy", "vinf"):
        assert rel_err(st[k], getattr(s, k)) <= TOL, k
    g.close()


def test_ensemble_members_with_fields(torch_cuda):
    from paper_1307_4839_amd.solver import Ensemble, Solver
    wls = [with_fields(I.hillslope_8192(150, 90), seed=6),
           I.ensemble_member(2, n=100),
           with_fields(I.hillslope_8192(70, 200), seed=7, soil=False)]
    e = Ensemble(wls)
    e.step(200)
    rc, flags = e.status()
    assert rc == 0
    for k, wl in enumerate(wls):
        g = Solver(wl)
        g.step(200)
        a, b = e.state(k), g.state()
        for f in b:
            assert np.array_equal(a[f], b[f]), (k, f)
        g.close()
    e.close()


def test_hyetograph_argument_checks(torch_cuda):
    from paper_1307_4839_amd import capi
    from paper_1307_4839_amd.solver import Solver
    g = Solver(I.hillslope_8192(40, 30))
    bad = [([0.0, 0.0], [1e-6, 1e-6]),           # not strictly increasing
           ([0.0, 5.0, 2.0], [0.0, 0.0, 0.0]),
           ([0.0], [-1e-6]),                     # negative rain
           ([math.nan], [1e-6]),
           ([0.0], [math.inf]),
           (list(range(capi.SWE_HYETO_MAX + 1)), [1e-6] * (capi.SWE_HYETO_MAX + 1))]
    for t_pts, r in bad:
        with pytest.raises(capi.SweError) as e:
            g.set_hyetograph(t_pts, r)
        assert e.value.code == capi.SWE_EINVAL
    # the largest table is accepted
    n = capi.SWE_HYETO_MAX
    g.set_hyetograph(np.arange(n, dtype=float), np.full(n, 1e-6))
    g.step(2)
    assert g.status()[0] == 0
    g.close()
