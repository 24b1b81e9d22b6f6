"""The collapse of the time step (eq. cfl) below dt_min, through the C ABI:
the step is not taken, the sticky DT_UNDERFLOW flag is raised and
swe_get_status returns SWE_EDTMIN; the last step of a run, clipped to the
end time, is exempt.  The GPU stops at the same step as the oracle with the
same state."""

import math
import sys

import numpy as np
import pytest

import oracle
from paper_1307_4839_amd import inputs as I

pytestmark = pytest.mark.gpu

G = 9.81


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def capi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1307_4839_amd import capi as c
    return c


def uniform(dt_min):
    h, u, v, dx, dy = 0.8, 0.9, -0.3, 2.0, 1.5
    z = np.zeros((7, 9))
    wl = I.Workload("uniform", 9, 7, dx, dy, z=z, h=z + h, qx=z + h * u, qy=z + h * v,
                    bc=(1, 1, 1, 1), dt_min=dt_min)
    c = math.sqrt(G * h)
    return wl, 0.5 / ((abs(u) + c) / dx + (abs(v) + c) / dy)


def test_dt_min_above_the_cfl_step(capi):
    from paper_1307_4839_amd.solver import Solver
    wl, dt = uniform(0.0)
    wl.dt_min = 1.01 * dt
    say("[dt_min] uniform 9x7, dt_min above the CFL step")
    g = Solver(wl)
    g.step(5)
    rc, flags = g.status()
    assert rc == capi.SWE_EDTMIN and flags == capi.SWE_FLAG_DT_UNDERFLOW
    t, _, steps = g.time()
    assert steps == 0 and t == 0.0
    st = g.state()
    assert np.array_equal(st["h"], wl.h) and np.array_equal(st["qx"], wl.qx)
    assert np.array_equal(st["qy"], wl.qy)
    g.close()


def test_dt_min_final_clipped_step_is_exempt(capi):
    from paper_1307_4839_amd.solver import Solver
    wl, dt = uniform(0.0)
    wl.dt_min = 0.99 * dt
    say("[dt_min] uniform 9x7, clipped last step")
    s = oracle.State(wl)
    assert s.run(10, 2.5 * dt) == 1 and s.steps == 3
    g = Solver(wl, dt_log=8)
    g.step(10, 2.5 * dt)
    rc, flags = g.status()
    assert rc == 0 and flags == 0
    t, _, steps = g.time()
    assert steps == 3 and t == s.t
    assert np.array_equal(g.dts(3), np.array(s.dts))
    g.close()


@pytest.mark.parametrize("order", [2, 1])
def test_dt_min_collapse_mid_run_matches_oracle(capi, order):
    from paper_1307_4839_amd.solver import Solver
    wl = I.dam_break_200(90, 70)
    # Darcy-Weisbach friction: every operation correctly rounded on both
    # sides, so the runs agree bit for bit
    wl.fric_law, wl.fric_coef = I.FRIC_DARCY, 0.2
    if order == 1:
        wl.order, wl.cfl = 1, 1.0
    free = oracle.State(wl)
    assert free.run(60) == 0
    dts = np.array(free.dts)
    k = 25
    wl.dt_min = 0.5 * (dts[:k].min() + dts[k:].min()) if dts[k:].min() < dts[:k].min() \
        else None
    assert wl.dt_min is not None, "the dam break's time step must shrink"
    s = oracle.State(wl)
    rc = s.run(60)
    assert rc == -5 and 0 < s.steps < 60
    say(f"[dt_min] dam break 90x70 order {order}: collapse after {s.steps} steps")
    g = Solver(wl, dt_log=64)
    g.step(60)
    rc_g, flags = g.status()
    assert rc_g == capi.SWE_EDTMIN and flags == capi.SWE_FLAG_DT_UNDERFLOW
    t, _, steps = g.time()
    assert steps == s.steps and t == s.t
    assert np.array_equal(g.dts(steps), np.array(s.dts))
    st = g.state()
    for f in ("h", "qx", "qy"):
        assert np.abs(st[f] - getattr(s, f)).max() <= 1e-12 * np.abs(getattr(s, f)).max(), f
    g.close()


def test_dt_min_in_an_ensemble_member(capi):
    from paper_1307_4839_amd.solver import Ensemble
    a, dt = uniform(0.0)
    b, _ = uniform(0.0)
    a.dt_min = 1.01 * dt
    say("[dt_min] ensemble of 2 uniform members, one collapsing")
    e = Ensemble([a, b])
    e.step(4)
    rc, flags = e.status()
    assert rc == capi.SWE_EDTMIN
    assert list(flags) == [capi.SWE_FLAG_DT_UNDERFLOW, 0]
    assert e.time(0)[2] == 0 and e.time(1)[2] == 4
    e.close()
