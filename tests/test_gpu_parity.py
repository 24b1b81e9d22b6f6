"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Bar: per field, max|gpu - oracle| / max|oracle| <= 1e-12 and
every step's dt within 1e-12 relative.  The kernels evaluate the formulas in
the oracle's order without contraction, so most cases agree bit for bit;
the bar stays the stated tolerance because the Manning cube root is not
correctly rounded on either side.
"""

import math
import sys

import numpy as np
import pytest

import oracle
from paper_1307_4839_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12


def rel_err(a, b):
    scale = max(np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() / scale


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def gpu_solver(wl, dt_log=0):
    from paper_1307_4839_amd.solver import Solver
    return Solver(wl, dt_log=dt_log)


def compare_run(wl, nsteps, t_end=math.inf, tol=TOL):
    say(f"[parity] {wl.name} {wl.nx}x{wl.ny} steps={nsteps}")
    s = oracle.State(wl)
    rc = s.run(nsteps, t_end)
    assert rc in (0, 1), rc
    g = gpu_solver(wl, dt_log=max(nsteps, 1))
    g.step(nsteps, t_end)
    t, last, steps = g.time()
    rc_g, flags = g.status()
    assert rc_g == 0 and flags == 0, (rc_g, flags)
    assert steps == s.steps
    st = g.state()
    errs = {k: rel_err(st[k], getattr(s, k)) for k in ("h", "qx", "qy")}
    if s.vinf is not None:
        errs["vinf"] = rel_err(st["vinf"], s.vinf)
    dts = g.dts()
    dt_err = np.abs(dts - np.array(s.dts)).max() / max(max(s.dts), 1e-300) if s.dts else 0.0
    same = int(np.array_equal(st["h"], s.h) and np.array_equal(st["qx"], s.qx)
               and np.array_equal(st["qy"], s.qy))
    say(f"    errs={errs} dt_err={dt_err:.3e} bitwise={same} t={t} oracle_t={s.t}")
    for k, e in errs.items():
        assert e <= tol, (k, e)
    assert dt_err <= tol
    assert abs(t - s.t) <= tol * max(abs(s.t), 1.0)
    g.close()
    return s, st


# ---------------------------------------------------------------------------
# Single rate evaluation and single steps on random valid states
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(37, 29), (300, 41), (505, 70), (252, 9), (2, 2), (253, 3)])
@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 1, 1, 1), (0, 1, 1, 0)])
def test_rate_random_state(torch_cuda, shape, bc):
    torch = torch_cuda
    nx, ny = shape
    wl = I.random_state(nx, ny, seed=nx * 7 + ny, bc=bc, dx=1.5, dy=0.7)
    say(f"[rate] {nx}x{ny} bc={bc}")
    p = oracle.params_of(wl)
    ph, pqx, pqy, amax = oracle.rate(p, wl.h, wl.qx, wl.qy, wl.z)
    g = gpu_solver(wl)
    gph, gpqx, gpqy, gam = g.rate(g.h, g.qx, g.qy)
    torch.cuda.synchronize()
    for a, b in ((gph, ph), (gpqx, pqx), (gpqy, pqy)):
        assert rel_err(a.cpu().numpy(), b) <= 1e-14
    assert gam[0] == amax[0] and gam[1] == amax[1]
    g.close()


@pytest.mark.parametrize("law,coef", [(0, 0.0), (1, 0.03), (2, 0.25)])
def test_single_step_random_state(torch_cuda, law, coef):
    wl = I.random_state(261, 77, seed=3 + law, bc=(0, 1, 1, 0), fric_law=law,
                        fric_coef=coef)
    compare_run(wl, 1, tol=1e-14)


def test_two_steps_rain_infiltration(torch_cuda):
    wl = I.random_state(130, 66, seed=17, bc=(1, 0, 0, 1), fric_law=2,
                        fric_coef=0.3, rain=1e-3, infil_on=1, ks=1e-5,
                        psi=0.1, dtheta=0.4)
    rng = np.random.default_rng(4)
    wl.vinf = rng.uniform(0, 1e-3, (wl.ny, wl.nx)) * (rng.uniform(0, 1, (wl.ny, wl.nx)) > 0.3)
    compare_run(wl, 2, tol=1e-14)


# ---------------------------------------------------------------------------
# Workload runs at oracle-friendly sizes (several tiles and ragged tails)
# ---------------------------------------------------------------------------

def test_dam_break_200_to_30s(torch_cuda):
    wl = I.dam_break_200()
    s, st = compare_run(wl, 100000, t_end=wl.t_end)
    assert s.t == 30.0


def test_valley_small(torch_cuda):
    wl = I.valley_2048(520, 600, dam_row=90)
    compare_run(wl, 300)


def test_hillslope_small_rain_infiltration(torch_cuda):
    wl = I.hillslope_8192(300, 260)
    s, st = compare_run(wl, 400)
    assert (s.h > 0).any()


@pytest.mark.parametrize("n", [100, 131])
def test_thacker_planar_one_period(torch_cuda, n):
    # a rotating plane surface in a paraboloid with its moving shoreline
    # (frictionless, walls far away): one full period, 131 cells a side
    # leaving ragged tiles; the results must be bitwise the oracle's
    wl = I.thacker_planar(n)
    s, st = compare_run(wl, wl.nsteps, t_end=wl.t_end, tol=0.0)
    assert s.t == wl.t_end


def test_calibration_small_friction_field(torch_cuda):
    wl = I.calibration_1024(260, 300, dam_row=40, ngauges=8, sigma_cells=6)
    compare_run(wl, 200)


def test_ensemble_member_small(torch_cuda):
    wl = I.ensemble_member(3, n=140)
    wl.rain = 3e-3  # wet it up quickly
    compare_run(wl, 150)


# ---------------------------------------------------------------------------
# Properties and edge cases
# ---------------------------------------------------------------------------

def test_lake_at_rest_on_gpu(torch_cuda):
    from test_oracle_pins import _islands
    C = 1.2
    wl = _islands(300, 90, C, seed=11, bc=(0, 1, 1, 0))
    g = gpu_solver(wl)
    g.step(500)
    st = g.state()
    wet = wl.h > 0
    assert np.abs((st["h"] + wl.z)[wet] - C).max() <= 1e-12 * C
    assert np.all(st["h"][~wet] == 0)
    H = wl.h.max()
    assert np.abs(st["qx"]).max() <= 1e-12 * math.sqrt(9.81 * H ** 3)
    assert np.abs(st["qy"]).max() <= 1e-12 * math.sqrt(9.81 * H ** 3)


def test_restart_bit_identical_gpu(torch_cuda):
    wl = I.hillslope_8192(200, 150)
    wl.rain = 200 * I.MM_PER_HOUR
    a = gpu_solver(wl)
    a.step(61)
    sa = a.state()
    b = gpu_solver(wl)
    b.step(30)
    sb = b.state()
    tb = b.time()[0]
    w2 = wl.copy()
    w2.h, w2.qx, w2.qy, w2.vinf = sb["h"], sb["qx"], sb["qy"], sb["vinf"]
    c = gpu_solver(w2)
    c.set_time(tb)
    c.step(31)
    sc = c.state()
    for k in ("h", "qx", "qy", "vinf"):
        assert np.array_equal(sa[k], sc[k]), k
    assert a.time()[0] == c.time()[0]


def test_run_to_run_bit_identical(torch_cuda):
    # the same run twice (thousands of blocks racing on the wave-speed
    # accumulators, graph replays) gives the same bits, for every flux
    for flux in (0, 1, 2):
        wl = I.hillslope_8192(1500, 1100)
        wl.rain = 150 * I.MM_PER_HOUR
        wl.flux = flux
        runs = []
        for _ in range(2):
            g = gpu_solver(wl)
            g.step(330)
            runs.append((g.state(), g.time()))
            g.close()
        (sa, ta), (sb, tb) = runs
        assert ta == tb
        for k in ("h", "qx", "qy", "vinf"):
            assert np.array_equal(sa[k], sb[k]), (flux, k)


def test_stop_at_t_end_and_odd_even_steps(torch_cuda):
    wl = I.dam_break_200(60, 50)
    s = oracle.State(wl)
    s.run(1000, 2.0)
    g = gpu_solver(wl)
    for k in (1, 2, 3, 5, 7, 1000):
        g.step(k, 2.0)
    t, _, steps = g.time()
    assert t == 2.0 and steps == s.steps
    st = g.state()
    assert rel_err(st["h"], s.h) <= TOL and rel_err(st["qx"], s.qx) <= TOL


def test_diagnostics(torch_cuda):
    wl = I.hillslope_8192(180, 120)
    wl.rain = 300 * I.MM_PER_HOUR
    g = gpu_solver(wl)
    g.step(50)
    d = g.diagnostics()
    st = g.state()
    assert abs(d.mass - st["h"].sum()) <= 1e-12 * max(st["h"].sum(), 1e-300)
    assert abs(d.infiltrated - st["vinf"].sum()) <= 1e-12 * st["vinf"].sum()
    assert d.h_min == st["h"].min() and d.h_max == st["h"].max()
    assert d.wet_cells == int((st["h"] > 1e-12).sum())


def _rain_rate(t_pts, r_pts, t):
    # the hyetograph: the value of the last breakpoint at or before t
    k = np.searchsorted(np.asarray(t_pts), t, side="right")
    return 0.0 if k == 0 else float(r_pts[k - 1])


@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (0, 1, 0, 0)])
def test_rain_in_and_outflow(torch_cuda, bc):
    # rain fallen = sum of dt r(t) over the steps times the summed weight;
    # outflow = the water balance; a walled basin loses nothing
    wl = I.hillslope_8192(130, 90)
    wl.bc = bc
    rng = np.random.default_rng(4)
    wl.rain_t = np.array([0.0, 40.0, 90.0])
    wl.rain_r = np.array([200.0, 20.0, 120.0]) * I.MM_PER_HOUR
    wl.rain_w = rng.uniform(0.5, 1.5, (wl.ny, wl.nx))
    s = oracle.State(wl)
    assert s.run(300) == 0
    g = gpu_solver(wl)
    g.step(300)
    d = g.diagnostics()
    area = wl.dx * wl.dy
    t, depth = 0.0, 0.0
    for dt in s.dts:
        depth += dt * _rain_rate(wl.rain_t, wl.rain_r, t)
        t += dt
    rain_in = depth * wl.rain_w.sum() * area
    assert abs(d.rain_in - rain_in) <= 1e-12 * rain_in
    water0 = (wl.h.sum() + wl.vinf.sum()) * area
    water = (s.h.sum() + s.vinf.sum()) * area
    out = water0 + rain_in - water
    assert abs(d.outflow - out) <= 1e-10 * (water0 + rain_in)
    if bc[1] == 0:
        assert abs(d.outflow) <= 1e-10 * (water0 + rain_in)
    else:
        assert d.outflow > 1e-3 * rain_in


def test_status_flags(torch_cuda):
    from paper_1307_4839_amd import capi
    # non-finite input poisons dt and the state: sticky flag
    wl = I.dam_break_200(40, 30)
    wl.h[5, 5] = float("nan")
    g = gpu_solver(wl)
    g.step(2)
    rc, flags = g.status()
    assert flags != 0 and rc in (capi.SWE_ENONFINITE, capi.SWE_EDT)
    # all dry, no rain, no dt bound, no final time: dt is not finite
    wl = I.dam_break_200(40, 30)
    wl.h[:] = 0
    g = gpu_solver(wl)
    g.step(1)
    rc, flags = g.status()
    assert rc == capi.SWE_EDT and flags & capi.SWE_FLAG_DT
    assert g.time()[2] == 0
    # a negative depth handed in is reported, never clamped
    wl = I.dam_break_200(40, 30)
    wl.h[3, 35] = -1e-3  # inside the dry half: no inflow reaches it
    wl.dt_max = 0.01
    g = gpu_solver(wl)
    g.step(1)
    rc, flags = g.status()
    assert flags & capi.SWE_FLAG_NEGDEPTH and rc == capi.SWE_ENEGDEPTH
    assert g.state()["h"][3, 35] < 0


def test_invalid_arguments(torch_cuda):
    from paper_1307_4839_amd import capi
    wl = I.dam_break_200(20, 20)
    g = gpu_solver(wl)
    with pytest.raises(capi.SweError):
        capi.swe_step(g.ctx, -1, 1.0)
    with pytest.raises(capi.SweError):
        capi.swe_set_rain(g.ctx, -1.0)


# ---------------------------------------------------------------------------
# Division paths.  The kernels share the reciprocal of a denominator among
# its quotients while the operands stay inside a window where this gives the
# division operator's value, and fall back to IEEE division for the rest of
# a tile (or for one lane's tail) otherwise.  Each case forces one path and
# must still match the oracle bit for bit (Darcy-Weisbach friction: every
# operation correctly rounded on both sides).
# ---------------------------------------------------------------------------

def _fallback_case(case):
    if case == "g_outside_window":
        # g > 2^10: every tile uses IEEE division from its first row
        return I.random_state(261, 77, seed=31, fric_law=2, fric_coef=0.3, g=2048.0)
    if case == "tiny_depth_mid_tile":
        # a wet cell of depth 1e-200 (h_eps = 0): the fast march of its tile
        # stops two rows before it and the tile ends in IEEE division
        wl = I.random_state(261, 150, seed=32, fric_law=2, fric_coef=0.3, h_eps=0.0)
        wl.h[100, 50], wl.qx[100, 50], wl.qy[100, 50] = 1e-200, 3e-201, -2e-201
        return wl
    if case == "huge_bed":
        wl = I.random_state(261, 150, seed=33, fric_law=2, fric_coef=0.3)
        wl.z[70, 120] += 1e70
        return wl
    if case == "negative_depth":
        wl = I.random_state(261, 150, seed=34, fric_law=2, fric_coef=0.3)
        wl.h[60, 40] = -1e-3
        return wl
    if case == "non_pow2_cells":
        return I.random_state(261, 150, seed=35, fric_law=2, fric_coef=0.3, dx=1.5, dy=0.7,
                              rain=1e-3, infil_on=1, ks=1e-5, psi=0.1, dtheta=0.4)
    raise ValueError(case)


@pytest.mark.parametrize("tx", [256, 64])
@pytest.mark.parametrize("case", ["g_outside_window", "tiny_depth_mid_tile", "huge_bed",
                                  "negative_depth", "non_pow2_cells"])
def test_division_paths(torch_cuda, case, tx):
    # tx 256: LDS exchange, block-wide flag; tx 64: DPP exchange, wave vote
    wl = _fallback_case(case)
    wl.dt_max = 0.01
    say(f"[division] {case} tiles {tx}")
    s = oracle.State(wl)
    s.run(1)
    g = gpu_solver(wl, dt_log=1)
    g.set_tiling(tx, 8)
    g.step(1)
    st = g.state()
    for k in ("h", "qx", "qy"):
        assert np.array_equal(st[k], getattr(s, k)), k
    assert np.array_equal(g.dts(), np.array(s.dts))
    g.close()
