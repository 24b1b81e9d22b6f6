"""swe_run_noalloc (the entry point for callers that cannot allocate device
memory) against swe_create + swe_set_time + swe_step on the same inputs,
through the C ABI: two calls in a row, the second on a smaller grid, each
bit for bit equal to the context's run (state, V_inf, time, last dt, steps,
flags); a grid above the scratch array's limit is refused."""

import math
import sys

import numpy as np
import pytest

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


def hillslope(nx, ny):
    wl = I.hillslope_8192(nx, ny)
    wl.rain = 2e-4  # ponds within a few tens of steps
    return wl


def run_noalloc(torch, wl, t0, nsteps, t_end):
    from paper_1307_4839_amd import capi
    from paper_1307_4839_amd.solver import _attach_fields, _dev, params_from
    dev = torch.device("cuda:0")
    h, qx, qy, z = (_dev(a, dev) for a in (wl.h, wl.qx, wl.qy, wl.z))
    vinf = _dev(wl.vinf if wl.vinf is not None else np.zeros_like(wl.h), dev) \
        if wl.infil_on else None
    fric = _dev(wl.fric, dev) if wl.fric is not None else None
    b = capi.swe_buffers()
    b.h, b.qx, b.qy, b.z = h.data_ptr(), qx.data_ptr(), qy.data_ptr(), z.data_ptr()
    b.fric = fric.data_ptr() if fric is not None else None
    b.vinf = vinf.data_ptr() if vinf is not None else None
    keep = _attach_fields(b, wl, dev)
    info = torch.full((4,), -1.0, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc = capi.swe_run_noalloc(params_from(wl), b, t0, nsteps, t_end, stream, info.data_ptr())
    assert rc == 0, rc
    torch.cuda.synchronize(dev)
    del keep
    out = {"h": h.cpu().numpy(), "qx": qx.cpu().numpy(), "qy": qy.cpu().numpy()}
    if vinf is not None:
        out["vinf"] = vinf.cpu().numpy()
    return out, info.cpu().numpy()


def run_context(wl, t0, nsteps, t_end):
    from paper_1307_4839_amd.solver import Solver
    g = Solver(wl, device="cuda:0")
    g.set_time(t0)
    g.step(nsteps, t_end)
    t, last_dt, steps = g.time()
    rc, flags = g.status()
    st = g.state()
    g.close()
    return st, np.array([t, last_dt, float(steps), float(flags)])


def check_same(torch, wl, t0, nsteps, t_end):
    say(f"[noalloc] {wl.name} {wl.nx}x{wl.ny} t0={t0} nsteps={nsteps} t_end={t_end}")
    a, ia = run_noalloc(torch, wl, t0, nsteps, t_end)
    b, ib = run_context(wl, t0, nsteps, t_end)
    assert np.array_equal(ia, ib), (ia, ib)
    for k in b:
        if k in a:
            assert np.array_equal(a[k], b[k]), k
    return ia


def test_noalloc_equals_swe_step_on_two_calls(torch_cuda):
    torch = torch_cuda
    # first call: the hillslope with rain, Green-Ampt and Darcy friction,
    # past ponding, an odd number of steps (the state ends in the scratch
    # array and is copied back)
    i1 = check_same(torch, hillslope(300, 260), 100.0, 301, math.inf)
    assert i1[2] == 301 and i1[3] == 0.0
    # second call, smaller grid: the dam break with Manning friction, clipped
    # at its end time, so fewer steps are taken than asked for
    wl = I.dam_break_200(120, 90)
    i2 = check_same(torch, wl, 0.0, 400, 2.0)
    assert abs(i2[0] - 2.0) <= 1e-12 and 0 < i2[2] < 400 and i2[3] == 0.0


def test_noalloc_first_order_rusanov(torch_cuda):
    torch = torch_cuda
    wl = I.dam_break_200(96, 64)
    wl.order, wl.cfl, wl.flux = 1, 1.0, 1
    check_same(torch, wl, 0.5, 37, math.inf)


def test_noalloc_refuses_grids_above_its_limit(torch_cuda):
    torch = torch_cuda
    from paper_1307_4839_amd import capi
    wl = I.dam_break_200(1025, 1024)
    assert wl.nx * wl.ny > capi.SWE_NOALLOC_MAX_CELLS
    p = capi.make_params(**wl.params())
    b = capi.swe_buffers()
    x = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    b.h = b.qx = b.qy = b.z = x.data_ptr()
    rc = capi.swe_run_noalloc(p, b, 0.0, 1, math.inf, None, x.data_ptr())
    assert rc == capi.SWE_ENOMEM
