"""GPU parity of the imposed boundaries (Section 2.2: depth, inflow
discharge or both imposed, the ghost from the Riemann invariants) with the
oracle, through the C ABI: single rates on random states with every type on
every side (fluvial, torrential and dry boundary cells), whole runs of the
channel over a bump on all four sides, at both orders and with the three
fluxes, torrential inflow into a dry channel, a 2D valley with rain fields,
tile-shape invariance, and ensemble members bit-identical to their own
runs."""

import math
import sys

import numpy as np
import pytest

import oracle
from paper_1307_4839_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12
H, Q, HQ = I.IMPOSED_H, I.IMPOSED_Q, I.IMPOSED_HQ


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


def compare(wl, nsteps, t_end=math.inf, tiling=None):
    from paper_1307_4839_amd.solver import Solver
    say(f"[imposed] {wl.name} {wl.nx}x{wl.ny} bc={wl.bc} order={wl.order} flux={wl.flux} "
        f"steps={nsteps} tiling={tiling}")
    s = oracle.State(wl)
    assert s.run(nsteps, t_end) in (0, 1)
    g = Solver(wl, dt_log=s.steps + 1)
    if tiling:
        g.set_tiling(*tiling)
    # a run to t_end: two steps more than the oracle took (steps past t_end
    # are no-ops; the step count is checked below)
    g.step(min(nsteps, s.steps + 2), t_end)
    rc, flags = g.status()
    assert rc == 0 and flags == 0, (rc, flags)
    # time steps: bitwise except through the Manning cube root (1 ulp)
    t, _, steps = g.time()
    assert steps == s.steps and abs(t - s.t) <= TOL * max(s.t, 1.0)
    assert np.abs(g.dts()[:steps] - np.array(s.dts)).max() <= TOL * max(s.dts)
    st = g.state()
    for k in ("h", "qx", "qy", "vinf"):
        if k in st:
            e = rel_err(st[k], getattr(s, k))
            say(f"    {k}: rel err {e:.3e} bitwise={np.array_equal(st[k], getattr(s, k))}")
            assert e <= TOL, k
    g.close()
    return s, st


def bump(nx, ny=4, q0=4.42, hb=2.0, axis="x", flip=False, **kw):
    """The 25 m channel over a parabolic bump: discharge q0 imposed
    upstream, depth hb downstream, walls on the sides; along x or y,
    flowing towards +axis or (flip) -axis."""
    d = 25.0 / nx
    x = (np.arange(nx) + 0.5) * d
    z1 = np.where((x > 8) & (x < 12), 0.2 - 0.05 * (x - 10) ** 2, 0.0)
    if flip:
        z1 = z1[::-1].copy()
    lo, hi = ((H, hb, 0.0), (Q, 0.0, q0)) if flip else ((Q, 0.0, q0), (H, hb, 0.0))
    if axis == "x":
        z = np.tile(z1, (ny, 1))
        bc, bch, bcq = (lo[0], hi[0], 0, 0), (lo[1], hi[1], 0, 0), (lo[2], hi[2], 0, 0)
        shape = (ny, nx)
    else:
        z = np.tile(z1[:, None], (1, ny))
        bc, bch, bcq = (0, 0, lo[0], hi[0]), (0, 0, lo[1], hi[1]), (0, 0, lo[2], hi[2])
        shape = (nx, ny)
    h = hb - z
    wl = I.Workload(f"bump_{axis}{'_flip' if flip else ''}", shape[1], shape[0], d, d, z=z, h=h,
                    qx=np.zeros(shape), qy=np.zeros(shape), bc=bc, bc_h=bch, bc_q=bcq, **kw)
    return wl


BC_MIXES = [((H, Q, HQ, H), (1.2, 0.0, 0.4, 0.9), (0.0, 1.5, 2.5, 0.0)),
            ((Q, H, Q, HQ), (0.0, 0.7, 0.0, 1.8), (0.8, 0.0, 0.0, 0.3)),
            ((HQ, 1, H, 0), (0.05, 0.0, 1.0, 0.0), (0.9, 0.0, 0.0, 0.0))]


@pytest.mark.parametrize("order", [2, 1])
@pytest.mark.parametrize("flux", [0, 1, 2])
@pytest.mark.parametrize("mix", range(len(BC_MIXES)))
@pytest.mark.parametrize("shape", [(37, 29), (300, 41), (2, 2)])
def test_rate_random_state(torch_cuda, shape, mix, flux, order):
    # random states put fluvial, torrential (1 mm films moving at 2 m/s)
    # and dry cells on the boundaries: every branch of the ghost
    from paper_1307_4839_amd.solver import Solver
    nx, ny = shape
    bc, bch, bcq = BC_MIXES[mix]
    wl = I.random_state(nx, ny, seed=nx * 5 + ny + mix, bc=bc, bc_h=bch, bc_q=bcq,
                        order=order, flux=flux)
    p = oracle.params_of(wl)
    ph, pqx, pqy, amax = oracle.rate(p, wl.h, wl.qx, wl.qy, wl.z)
    g = Solver(wl)
    gph, gpqx, gpqy, gamax = g.rate(g.h, g.qx, g.qy)
    torch_cuda.cuda.synchronize()
    for a, b in ((gph, ph), (gpqx, pqx), (gpqy, pqy)):
        assert np.array_equal(a.cpu().numpy(), b)
    assert gamax[0] == amax[0] and gamax[1] == amax[1]
    g.close()


@pytest.mark.parametrize("axis,flip", [("x", False), ("x", True), ("y", False), ("y", True)])
def test_bump_every_side(torch_cuda, axis, flip):
    compare(bump(100, axis=axis, flip=flip), 10 ** 6, t_end=20.0)


@pytest.mark.parametrize("order,flux", [(1, 0), (2, 1), (1, 1), (2, 2), (1, 2)])
def test_bump_scheme_variants(torch_cuda, order, flux):
    compare(bump(100, order=order, flux=flux, cfl=1.0 if order == 1 else 0.5), 1500)


def test_bump_to_steady_state_against_bernoulli(torch_cuda):
    # long run: the GPU run reaches the steady Bernoulli profile exactly as
    # the oracle does
    s, st = compare(bump(200, ny=3), 10 ** 6, t_end=120.0)
    assert np.abs(st["qx"] - 4.42).max() <= 0.02


@pytest.mark.parametrize("tiling", [None, (64, 8), (128, 16), (256, 4)])
def test_tile_shapes(torch_cuda, tiling):
    # 300 columns: the east ghosts fall in the middle of a strip for some
    # widths and at a strip edge for others
    wl = bump(300, ny=37)
    wl.bc = (Q, H, Q, H)
    wl.bc_h = (0.0, 2.0, 0.0, 2.1)
    wl.bc_q = (4.42, 0.0, 0.3, 0.0)
    compare(wl, 300, tiling=tiling)


def test_torrential_inflow_into_dry_channel(torch_cuda):
    z = np.zeros((3, 120))
    wl = I.Workload("torrent", 120, 3, 0.5, 0.5, z=z, h=z.copy(), qx=z.copy(), qy=z.copy(),
                    bc=(HQ, H, 0, 0), bc_h=(0.5, 0.4, 0, 0), bc_q=(5.0, 0, 0, 0),
                    fric_law=I.FRIC_MANNING, fric_coef=0.02)
    compare(wl, 10 ** 6, t_end=15.0)


def test_valley_with_rain_fields_and_imposed_sides(torch_cuda):
    # the FIELDS variant with imposed sides: a valley fed through its north
    # side, a fixed level on the south, hyetograph and weighted rain
    wl = I.valley_2048(160, 190, dam_row=40)
    rng = np.random.default_rng(12)
    wl.bc = (0, 0, H, Q)
    wl.bc_h = (0.0, 0.0, 0.5, 0.0)
    wl.bc_q = (0.0, 0.0, 0.0, 0.2)
    wl.rain_t = np.array([0.0, 5.0, 12.0])
    wl.rain_r = np.array([100.0, 300.0, 50.0]) * I.MM_PER_HOUR
    wl.rain_w = rng.uniform(0.5, 1.5, (wl.ny, wl.nx))
    compare(wl, 400)


def test_ensemble_members_with_imposed_sides(torch_cuda):
    # members with imposed sides (and one without) evolve in the ensemble
    # exactly as in their own contexts
    from paper_1307_4839_amd.solver import Ensemble, Solver
    v = I.valley_2048(90, 110, dam_row=30)
    v.bc, v.bc_h, v.bc_q = (0, 0, H, Q), (0.0, 0.0, 0.5, 0.0), (0.0, 0.0, 0.0, 0.2)
    v.rain_w = np.random.default_rng(5).uniform(0.5, 1.5, (v.ny, v.nx))
    wls = [bump(120, ny=9), I.ensemble_member(2, n=100), v, bump(70, ny=5, axis="y", flip=True)]
    e = Ensemble(wls)
    e.step(200)
    rc, _ = e.status()
    assert rc == 0
    for k, wl in enumerate(wls):
        g = Solver(wl)
        g.step(200)
        a, b = e.state(k), g.state()
        for f in b:
            assert np.array_equal(a[f], b[f]), (k, f)
        g.close()
    e.close()


def test_hydrograph_by_boundary_value_updates(torch_cuda):
    # the inflow discharge and the outlet level changed between calls of
    # swe_step (a stepwise hydrograph): the same as the oracle with the
    # parameters changed at the same steps, in a context and in an ensemble
    from paper_1307_4839_amd import capi
    from paper_1307_4839_amd.solver import Ensemble, Solver
    wl = bump(120, ny=5)
    plan = [(200, 4.42, 2.0), (150, 3.1, 1.9), (170, 5.0, 2.05)]
    s = oracle.State(wl)
    g = Solver(wl, dt_log=600)
    e = Ensemble([wl, I.ensemble_member(1, n=80)])
    for n, q, h in plan:
        w2 = wl.copy()
        w2.bc_q, w2.bc_h = (q, 0, 0, 0), (0, h, 0, 0)
        s.p = oracle.params_of(w2)
        assert s.run(n) == 0
        g.set_boundary_values(0, q_b=q)
        g.set_boundary_values(1, h_b=h)
        g.step(n)
        e.set_boundary_values(0, 0, q_b=q)
        e.set_boundary_values(0, 1, h_b=h)
        e.step(n)
    st = g.state()
    assert g.time()[2] == s.steps
    for k in ("h", "qx", "qy"):
        assert rel_err(st[k], getattr(s, k)) <= TOL, k
    es = e.state(0)
    for k in ("h", "qx", "qy"):
        assert np.array_equal(es[k], st[k]), k
    # the side must be imposed and the values valid for its type
    for side, hb, qb in ((2, 1.0, 0.0), (0, 0.0, -1.0), (1, 0.0, 0.0), (1, math.nan, 0.0),
                         (4, 1.0, 1.0)):
        with pytest.raises(capi.SweError) as err:
            g.set_boundary_values(side, h_b=hb, q_b=qb)
        assert err.value.code == capi.SWE_EINVAL
    with pytest.raises(capi.SweError):
        e.set_boundary_values(1, 0, q_b=1.0)     # member 1 has no imposed side
    g.close()
    e.close()
