"""GPU parity of the Rusanov and kinetic fluxes (two other consistent
fluxes Section 3.3 lists beside HLL) with the oracle, through the C ABI:
single rates on random states, whole runs at second and first order, with
rain, Green-Ampt and the optional fields, over several tile shapes."""

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


RUSANOV, KINETIC = 1, 2
FLUXES = pytest.mark.parametrize("flux", [RUSANOV, KINETIC])


def variant(wl, flux, order=2):
    wl = wl.copy()
    wl.flux = flux
    if order == 1:
        wl.order, wl.cfl = 1, 1.0
    return wl


def compare(wl, nsteps, t_end=math.inf, tiling=None):
    from paper_1307_4839_amd.solver import Solver
    say(f"[flux {wl.flux}] {wl.name} {wl.nx}x{wl.ny} order={wl.order} steps={nsteps} "
        f"tiling={tiling}")
    s = oracle.State(wl)
    assert s.run(nsteps, t_end) in (0, 1)
    g = Solver(wl, dt_log=s.steps + 1)
    if tiling:
        g.set_tiling(*tiling)
    g.step(min(nsteps, s.steps + 2), t_end)  # steps past t_end are no-ops
    rc, flags = g.status()
    assert rc == 0 and flags == 0, (rc, flags)
    _, _, steps = g.time()
    assert steps == s.steps
    assert np.abs(g.dts()[:steps] - np.array(s.dts)).max() <= TOL * max(s.dts)
    st = g.state()
    same = True
    for k in ("h", "qx", "qy", "vinf"):
        if k in st:
            e = rel_err(st[k], getattr(s, k))
            same = same and np.array_equal(st[k], getattr(s, k))
            assert e <= TOL, (k, e)
    say(f"    bitwise={same}")
    g.close()
    return s, st


@FLUXES
@pytest.mark.parametrize("order", [2, 1])
@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 1, 1, 1), (0, 1, 1, 0)])
@pytest.mark.parametrize("shape", [(37, 29), (300, 41), (2, 2)])
def test_rate_random_state(torch_cuda, shape, bc, order, flux):
    from paper_1307_4839_amd.solver import Solver
    nx, ny = shape
    wl = variant(I.random_state(nx, ny, seed=nx * 5 + ny, bc=bc, dx=1.5, dy=0.7), flux, order)
    p = oracle.params_of(wl)
    ph, pqx, pqy, amax = oracle.rate(p, wl.h, wl.qx, wl.qy, wl.z)
    g = Solver(wl)
    gph, gpqx, gpqy, gamax = g.rate(g.h, g.qx, g.qy)
    torch_cuda.cuda.synchronize()
    for a, b in ((gph, ph), (gpqx, pqx), (gpqy, pqy)):
        assert np.array_equal(a.cpu().numpy(), b)
    assert gamax[0] == amax[0] and gamax[1] == amax[1]
    g.close()


@FLUXES
@pytest.mark.parametrize("order", [2, 1])
def test_dam_break_200_to_30s(torch_cuda, order, flux):
    s, _ = compare(variant(I.dam_break_200(), flux, order), 10 ** 6, t_end=30.0)
    assert s.t == 30.0


@FLUXES
@pytest.mark.parametrize("tiling", [None, (64, 8), (128, 16)])
def test_hillslope_rain_infiltration(torch_cuda, tiling, flux):
    compare(variant(I.hillslope_8192(260, 200), flux), 400, tiling=tiling)


@FLUXES
def test_valley_first_order(torch_cuda, flux):
    compare(variant(I.valley_2048(300, 320, dam_row=60), flux, order=1), 300)


@FLUXES
def test_valley_second_order(torch_cuda, flux):
    compare(variant(I.valley_2048(300, 320, dam_row=60), flux), 300)


@FLUXES
def test_fields_and_hyetograph(torch_cuda, flux):
    wl = variant(I.hillslope_8192(200, 150), flux)
    rng = np.random.default_rng(9)
    wl.rain_t = np.array([0.0, 120.0])
    wl.rain_r = np.array([90.0, 30.0]) * I.MM_PER_HOUR
    wl.rain_w = rng.uniform(0.3, 1.7, (wl.ny, wl.nx))
    wl.psi_f = wl.psi * rng.uniform(0.5, 1.5, (wl.ny, wl.nx))
    compare(wl, 400)


@pytest.mark.parametrize("order,flux", [(1, 0), (1, 1), (1, 2), (2, 1), (2, 2)])
def test_ensemble_members_bit_identical(torch_cuda, order, flux):
    # ensembles whose members share a scheme variant: each member evolves as
    # in its own context (graph replays, an autotuned tiling, a member
    # with rain and soil fields, one with imposed sides)
    from paper_1307_4839_amd.solver import Ensemble, Solver
    rng = np.random.default_rng(order * 10 + flux)
    a = I.hillslope_8192(150, 90)
    a.rain_w = rng.uniform(0.5, 1.5, (a.ny, a.nx))
    a.ks_f = a.ks * rng.uniform(0.5, 1.5, (a.ny, a.nx))
    c = I.valley_2048(90, 110, dam_row=30)
    c.bc, c.bc_h, c.bc_q = (0, 0, I.IMPOSED_H, I.IMPOSED_Q), (0, 0, 0.5, 0), (0, 0, 0, 0.2)
    wls = [variant(w, flux, order) for w in (a, I.ensemble_member(3, n=100), c)]
    e = Ensemble(wls)
    if order == 1:
        e.autotune(4)
    e.step(150)
    rc, _ = e.status()
    assert rc == 0
    for k, wl in enumerate(wls):
        g = Solver(wl)
        g.step(150)
        a_, b_ = e.state(k), g.state()
        for f in b_:
            assert np.array_equal(a_[f], b_[f]), (k, f)
        g.close()
    e.close()
