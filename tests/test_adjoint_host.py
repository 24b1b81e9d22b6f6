"""Host (CPU) checks of the adjoint's reverse routines.

The per-face and per-cell functions of the adjoint are __host__ __device__;
tests/adjoint_host_emu.hip builds them for the CPU.  Checked against the
oracle (no GPU needed), with the HLL, Rusanov and kinetic fluxes:
  * the vector-Jacobian product of the convective rate equals central
    differences of the oracle's rate (three boundary mixes, ghost folding);
  * one full reverse step (Heun split, both frictions, both VJPs) gives
    <grad, d> equal to the oracle's forward-mode tangent to round-off.
"""

import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_1307_4839_amd import capi
from paper_1307_4839_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DP = C.POINTER(C.c_double)


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("emu") / "libadjemu.so")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC",
                           "-shared", "-ffp-contract=off", "-I", os.path.join(ROOT, "include"),
                           os.path.join(HERE, "adjoint_host_emu.hip"), "-o", out,
                           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
                           "-Wl,-rpath,/opt/rocm/lib"],
                          stderr=subprocess.DEVNULL)
    return C.CDLL(out)


def P(a):
    return np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(DP)


def vjp(L, cp, wl, U, mu):
    out = [np.zeros(U[0].shape) for _ in range(3)]
    L.emu_vjp(C.byref(cp), P(wl.z), P(U[0]), P(U[1]), P(U[2]), P(mu[0]), P(mu[1]), P(mu[2]),
              *[o.ctypes.data_as(DP) for o in out])
    return out


@pytest.mark.parametrize("flux", [0, 1, 2])
@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 1, 1, 1), (0, 1, 1, 0)])
def test_rate_vjp_matches_oracle_differences(emu, bc, flux):
    rng = np.random.default_rng(0)
    wl = I.random_state(23, 19, seed=4, bc=bc, dx=1.3, dy=0.8, dry_frac=0.0, film_frac=0.0,
                        flux=flux)
    p = oracle.params_of(wl)
    cp = capi.make_params(**wl.params())
    mu = [rng.standard_normal((wl.ny, wl.nx)) for _ in range(3)]
    out = vjp(emu, cp, wl, [wl.h, wl.qx, wl.qy], mu)
    d = [rng.standard_normal((wl.ny, wl.nx)) * 0.1 for _ in range(3)]
    eps = 1e-7
    rp = oracle.rate(p, wl.h + eps * d[0], wl.qx + eps * d[1], wl.qy + eps * d[2], wl.z)
    rm = oracle.rate(p, wl.h - eps * d[0], wl.qx - eps * d[1], wl.qy - eps * d[2], wl.z)
    lhs = sum(((rp[k] - rm[k]) / (2 * eps) * mu[k]).sum() for k in range(3))
    rhs = sum((out[k] * d[k]).sum() for k in range(3))
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)


@pytest.mark.parametrize("flux", [0, 1, 2])
@pytest.mark.parametrize("case", ["valley", "random"])
def test_one_reverse_step_matches_oracle_tangent(emu, case, flux):
    L = emu
    if case == "valley":
        wl = I.calibration_1024(40, 36, dam_row=10, ngauges=4, sigma_cells=3)
        wl.flux = flux
        s = oracle.State(wl)
        s.run(15)
        wl.h, wl.qx, wl.qy = s.h.copy(), s.qx.copy(), s.qy.copy()
    else:
        wl = I.random_state(30, 26, seed=3, bc=(1, 0, 0, 1), fric_law=1, fric_coef=0.04,
                            flux=flux)
        wl.fric = 0.04 * (1 + 0.2 * I.smooth_field(np.random.default_rng(2), 30, 26, 3.0))
    p = oracle.params_of(wl)
    cp = capi.make_params(**wl.params())
    shape = wl.h.shape
    Z = lambda: np.zeros(shape)
    dt = 0.5 * oracle.time_step(p, oracle.rate(p, wl.h, wl.qx, wl.qy, wl.z)[3], 0.0, np.inf)
    U = [wl.h, wl.qx, wl.qy]
    obs = np.random.default_rng(5).uniform(0, 1, shape)
    gauges = np.arange(wl.nx * wl.ny, dtype=np.int32)
    s1 = oracle.State(wl)
    s1.step_fixed(dt)
    lam = [2 * (s1.h - obs), Z(), Z()]
    ph1 = oracle.rate(p, *U, wl.z)[:3]
    Us = [Z() for _ in range(3)]
    L.emu_stage_out(C.byref(cp), P(wl.fric), *[P(a) for a in U], *[P(a) for a in ph1],
                    C.c_double(dt), *[a.ctypes.data_as(DP) for a in Us])
    lamA = [0.5 * l for l in lam]
    ph2 = oracle.rate(p, *Us, wl.z)[:3]
    lamB, mu, grad = [Z() for _ in range(3)], [Z() for _ in range(3)], Z()
    L.emu_adj_stage(C.byref(cp), P(wl.fric), *[P(a) for a in Us], *[P(a) for a in ph2],
                    C.c_double(dt), *[P(a) for a in lam], C.c_double(0.5),
                    *[a.ctypes.data_as(DP) for a in lamB], *[a.ctypes.data_as(DP) for a in mu],
                    grad.ctypes.data_as(DP))
    v = vjp(L, cp, wl, Us, mu)
    lamB = [lamB[k] + v[k] for k in range(3)]
    lin = [Z() for _ in range(3)]
    L.emu_adj_stage(C.byref(cp), P(wl.fric), *[P(a) for a in U], *[P(a) for a in ph1],
                    C.c_double(dt), *[P(a) for a in lamB], C.c_double(1.0),
                    *[a.ctypes.data_as(DP) for a in lin], *[a.ctypes.data_as(DP) for a in mu],
                    grad.ctypes.data_as(DP))
    rng = np.random.default_rng(1)
    for _ in range(3):
        d = rng.standard_normal(shape) * 1e-3
        _, dL = oracle.tangent_run(p, wl.h, wl.qx, wl.qy, wl.z, wl.fric, d, [dt], gauges, 1, obs)
        gd = (grad * d).sum()
        assert abs(gd - dL) <= 1e-12 * abs(dL)
