"""ctypes binding of the C ABI declared in ``include/swe.h`` and
``include/swe_flowdir.h``.

Argument marshalling only: every step of the method runs in the HIP
library.  If the library has not been built the import of this module
raises, so there is no silent fallback.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SWE_LIB") or os.path.join(_PKG, "libswe_mi355x.so")

SWE_OK = 0
SWE_EINVAL = -1
SWE_EHIP = -2
SWE_ENEGDEPTH = -3
SWE_ENONFINITE = -4
SWE_EDTMIN = -5
SWE_ENOMEM = -6
SWE_EDT = -7

SWE_FLAG_NEGDEPTH = 1
SWE_FLAG_NONFINITE = 2
SWE_FLAG_DT = 4
SWE_FLAG_DT_UNDERFLOW = 8

SWE_BC_WALL = 0
SWE_BC_OUTFLOW = 1
SWE_BC_IMPOSED_H = 2
SWE_BC_IMPOSED_Q = 3
SWE_BC_IMPOSED_HQ = 4
SWE_FRIC_NONE = 0
SWE_FRIC_MANNING = 1
SWE_FRIC_DARCY = 2
SWE_MAX_NX = 1 << 28  # longest row (cells along x)


class swe_params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double),
                ("g", C.c_double), ("cfl", C.c_double),
                ("dt_max", C.c_double), ("h_eps", C.c_double),
                ("bc", C.c_int32 * 4), ("fric_law", C.c_int32),
                ("fric_coef", C.c_double), ("rain", C.c_double),
                ("infil_on", C.c_int32), ("ks", C.c_double),
                ("psi", C.c_double), ("dtheta", C.c_double), ("order", C.c_int32),
                ("flux", C.c_int32), ("bc_h", C.c_double * 4), ("bc_q", C.c_double * 4),
                ("dt_min", C.c_double), ("recon", C.c_int32)]


class swe_buffers(C.Structure):
    _fields_ = [("h", C.c_void_p), ("qx", C.c_void_p), ("qy", C.c_void_p),
                ("z", C.c_void_p), ("fric", C.c_void_p), ("vinf", C.c_void_p),
                ("rain_w", C.c_void_p), ("ks", C.c_void_p), ("psi", C.c_void_p),
                ("dtheta", C.c_void_p)]


SWE_HYETO_MAX = 128


class swe_diag(C.Structure):
    _fields_ = [("mass", C.c_double), ("infiltrated", C.c_double),
                ("h_min", C.c_double), ("h_max", C.c_double),
                ("wet_cells", C.c_int64), ("rain_in", C.c_double),
                ("outflow", C.c_double)]


EXPORTS = {
    # name: (restype, argtypes)
    "swe_workspace_bytes": (C.c_int, [C.POINTER(swe_params), C.POINTER(C.c_size_t)]),
    "swe_create": (C.c_int, [C.POINTER(swe_params), C.POINTER(swe_buffers),
                             C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "swe_destroy": (C.c_int, [C.c_void_p]),
    "swe_run_noalloc": (C.c_int, [C.POINTER(swe_params), C.POINTER(swe_buffers), C.c_double,
                                  C.c_int32, C.c_double, C.c_void_p, C.c_void_p]),
    "swe_set_tiling": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "swe_get_tiling": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "swe_set_time": (C.c_int, [C.c_void_p, C.c_double]),
    "swe_set_rain": (C.c_int, [C.c_void_p, C.c_double]),
    "swe_set_hyetograph": (C.c_int, [C.c_void_p, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.c_int32]),
    "swe_set_dt_log": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "swe_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_double]),
    "swe_set_boundary_values": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_double]),
    "swe_batch_set_boundary_values": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_double,
                                                C.c_double]),
    "swe_set_gauges": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                 C.c_int64]),
    "swe_get_gauges": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]),
    "swe_get_time": (C.c_int, [C.c_void_p, C.POINTER(C.c_double),
                               C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "swe_get_status": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint32)]),
    "swe_get_diagnostics": (C.c_int, [C.c_void_p, C.POINTER(swe_diag)]),
    "swe_rate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                           C.c_void_p, C.c_void_p, C.c_void_p,
                           C.POINTER(C.c_double)]),
    "swe_profile_begin": (C.c_int, [C.c_void_p, C.c_int32]),
    "swe_profile_end": (C.c_int, [C.c_void_p, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "swe_batch_workspace_bytes": (C.c_int, [C.POINTER(swe_params), C.c_int32,
                                            C.POINTER(C.c_size_t)]),
    "swe_batch_create": (C.c_int, [C.POINTER(swe_params), C.POINTER(swe_buffers), C.c_int32,
                                   C.c_void_p, C.c_size_t, C.c_void_p,
                                   C.POINTER(C.c_void_p)]),
    "swe_batch_destroy": (C.c_int, [C.c_void_p]),
    "swe_batch_set_tiling": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "swe_batch_get_tiling": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "swe_batch_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "swe_batch_set_rain": (C.c_int, [C.c_void_p, C.c_int32, C.c_double]),
    "swe_batch_set_hyetograph": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                                           C.POINTER(C.c_double), C.c_int32]),
    "swe_batch_set_dt_log": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64]),
    "swe_batch_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_double]),
    "swe_batch_get_time": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "swe_batch_get_status": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint32), C.c_int32]),
    "swe_adj_workspace_bytes": (C.c_int, [C.POINTER(swe_params), C.c_int32, C.c_int32,
                                          C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "swe_adj_create": (C.c_int, [C.POINTER(swe_params), C.POINTER(swe_buffers), C.c_int32,
                                 C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                 C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "swe_adj_destroy": (C.c_int, [C.c_void_p]),
    "swe_adj_set_dts": (C.c_int, [C.c_void_p, C.c_void_p]),
    "swe_adj_get_dts": (C.c_int, [C.c_void_p, C.c_void_p]),
    "swe_adj_forward": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "swe_adj_backward": (C.c_int, [C.c_void_p, C.c_void_p]),
    "swe_adj_get_series": (C.c_int, [C.c_void_p, C.c_void_p]),
    "swe_flow_dir_f32": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                                   C.c_void_p]),
    "swe_flow_dir_f64": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                                   C.c_void_p]),
    "swe_flow_dir_rows": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]),
    "swe_strerror": (C.c_char_p, [C.c_int]),
}


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"HIP library {path} is not built; run "
            "`python -m paper_1307_4839_amd.build` (or __graft_entry__.build())")
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


class SweError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().swe_strerror(code).decode()
        super().__init__(f"{where}: {msg} ({code})")
        self.code = code


def check(code: int, where: str) -> int:
    if code != SWE_OK:
        raise SweError(code, where)
    return code


def make_params(nx, ny, dx, dy, g=9.81, cfl=0.5, dt_max=float("inf"),
                h_eps=1e-12, bc=(0, 0, 0, 0), fric_law=0, fric_coef=0.0,
                rain=0.0, infil_on=0, ks=0.0, psi=0.0, dtheta=0.0, order=2,
                flux=0, bc_h=(0.0,) * 4, bc_q=(0.0,) * 4, dt_min=0.0, recon=0) -> swe_params:
    p = swe_params()
    p.dt_min = float(dt_min)
    p.recon = int(recon)
    p.order = int(order)
    p.flux = int(flux)
    for k in range(4):
        p.bc_h[k] = float(bc_h[k])
        p.bc_q[k] = float(bc_q[k])
    p.nx, p.ny, p.dx, p.dy = nx, ny, dx, dy
    p.g, p.cfl, p.dt_max, p.h_eps = g, cfl, dt_max, h_eps
    for k in range(4):
        p.bc[k] = int(bc[k])
    p.fric_law, p.fric_coef, p.rain = int(fric_law), fric_coef, rain
    p.infil_on, p.ks, p.psi, p.dtheta = int(infil_on), ks, psi, dtheta
    return p


# Thin wrappers with the C names (pointers are ints / ctypes values)

def swe_workspace_bytes(p: swe_params) -> int:
    n = C.c_size_t(0)
    check(lib().swe_workspace_bytes(C.byref(p), C.byref(n)), "swe_workspace_bytes")
    return n.value


def swe_create(p: swe_params, b: swe_buffers, workspace: int, nbytes: int,
               stream: int) -> int:
    ctx = C.c_void_p(0)
    check(lib().swe_create(C.byref(p), C.byref(b), C.c_void_p(workspace), nbytes,
                           C.c_void_p(stream), C.byref(ctx)), "swe_create")
    return ctx.value


def swe_destroy(ctx: int) -> None:
    check(lib().swe_destroy(C.c_void_p(ctx)), "swe_destroy")


def swe_set_tiling(ctx: int, tx: int, ty: int = 0) -> None:
    check(lib().swe_set_tiling(C.c_void_p(ctx), tx, ty), "swe_set_tiling")


def swe_get_tiling(ctx: int):
    tx, ty = C.c_int32(), C.c_int32()
    check(lib().swe_get_tiling(C.c_void_p(ctx), C.byref(tx), C.byref(ty)), "swe_get_tiling")
    return tx.value, ty.value


def swe_set_time(ctx: int, t: float) -> None:
    check(lib().swe_set_time(C.c_void_p(ctx), t), "swe_set_time")


def swe_set_rain(ctx: int, rain: float) -> None:
    check(lib().swe_set_rain(C.c_void_p(ctx), rain), "swe_set_rain")


def _table(a):
    if a is None:
        return None, 0
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, len(a)


def swe_set_hyetograph(ctx: int, t_pts, r) -> None:
    """Host sequences (or None to remove the hyetograph)."""
    t_a, n = _table(t_pts)
    r_a, m = _table(r)
    if n != m:
        raise ValueError("t_pts and r differ in length")
    dp = C.POINTER(C.c_double)
    check(lib().swe_set_hyetograph(C.c_void_p(ctx),
                                   None if t_a is None else t_a.ctypes.data_as(dp),
                                   None if r_a is None else r_a.ctypes.data_as(dp), n),
          "swe_set_hyetograph")


def swe_batch_set_hyetograph(b: int, member: int, t_pts, r) -> None:
    t_a, n = _table(t_pts)
    r_a, m = _table(r)
    if n != m:
        raise ValueError("t_pts and r differ in length")
    dp = C.POINTER(C.c_double)
    check(lib().swe_batch_set_hyetograph(C.c_void_p(b), member,
                                         None if t_a is None else t_a.ctypes.data_as(dp),
                                         None if r_a is None else r_a.ctypes.data_as(dp), n),
          "swe_batch_set_hyetograph")


def swe_set_dt_log(ctx: int, ptr: int, capacity: int) -> None:
    check(lib().swe_set_dt_log(C.c_void_p(ctx), C.c_void_p(ptr), capacity),
          "swe_set_dt_log")


def swe_set_gauges(ctx: int, cells_ptr: int, ngauges: int, every: int, series_ptr: int,
                   max_samples: int) -> None:
    check(lib().swe_set_gauges(C.c_void_p(ctx), C.c_void_p(cells_ptr), ngauges, every,
                               C.c_void_p(series_ptr), max_samples), "swe_set_gauges")


def swe_get_gauges(ctx: int, out: Optional[np.ndarray] = None) -> int:
    """Samples recorded so far; fills out (float64, C-contiguous, rows of
    ngauges values) with as many as fit."""
    n = C.c_int64(0)
    if out is None:
        check(lib().swe_get_gauges(C.c_void_p(ctx), None, 0, C.byref(n)), "swe_get_gauges")
    else:
        assert out.dtype == np.float64 and out.flags.c_contiguous and out.ndim == 2
        check(lib().swe_get_gauges(C.c_void_p(ctx), out.ctypes.data_as(C.c_void_p),
                                   out.shape[0], C.byref(n)), "swe_get_gauges")
    return n.value


def swe_set_boundary_values(ctx: int, side: int, h_b: float, q_b: float) -> None:
    check(lib().swe_set_boundary_values(C.c_void_p(ctx), side, h_b, q_b),
          "swe_set_boundary_values")


def swe_batch_set_boundary_values(b: int, member: int, side: int, h_b: float,
                                  q_b: float) -> None:
    check(lib().swe_batch_set_boundary_values(C.c_void_p(b), member, side, h_b, q_b),
          "swe_batch_set_boundary_values")


def swe_step(ctx: int, nsteps: int, t_end: float = float("inf")) -> None:
    check(lib().swe_step(C.c_void_p(ctx), nsteps, t_end), "swe_step")


SWE_NOALLOC_MAX_CELLS = 1 << 20


def swe_run_noalloc(p: swe_params, b: swe_buffers, t0: float, nsteps: int, t_end: float,
                    stream: Optional[int], info: int) -> int:
    """Returns the status code (the caller checks it; no exception, so that
    a test can see SWE_ENOMEM)."""
    return lib().swe_run_noalloc(C.byref(p), C.byref(b), t0, nsteps, t_end,
                                 C.c_void_p(stream or 0), C.c_void_p(info))


def swe_get_time(ctx: int):
    t, dt, n = C.c_double(), C.c_double(), C.c_int64()
    check(lib().swe_get_time(C.c_void_p(ctx), C.byref(t), C.byref(dt), C.byref(n)),
          "swe_get_time")
    return t.value, dt.value, n.value


def swe_get_status(ctx: int):
    f = C.c_uint32(0)
    rc = lib().swe_get_status(C.c_void_p(ctx), C.byref(f))
    return rc, f.value


def swe_get_diagnostics(ctx: int) -> swe_diag:
    d = swe_diag()
    check(lib().swe_get_diagnostics(C.c_void_p(ctx), C.byref(d)), "swe_get_diagnostics")
    return d


def swe_rate(ctx: int, h: int, qx: int, qy: int, ph: int, pqx: int, pqy: int):
    amax = (C.c_double * 2)()
    check(lib().swe_rate(C.c_void_p(ctx), C.c_void_p(h), C.c_void_p(qx),
                         C.c_void_p(qy), C.c_void_p(ph), C.c_void_p(pqx),
                         C.c_void_p(pqy), amax), "swe_rate")
    return amax[0], amax[1]


def swe_profile_begin(ctx: int, max_steps: int) -> None:
    check(lib().swe_profile_begin(C.c_void_p(ctx), max_steps), "swe_profile_begin")


def swe_profile_end(ctx: int):
    a, b, n = C.c_double(), C.c_double(), C.c_int32()
    check(lib().swe_profile_end(C.c_void_p(ctx), C.byref(a), C.byref(b), C.byref(n)),
          "swe_profile_end")
    return a.value, b.value, n.value


# -- ensembles -----------------------------------------------------------------

def swe_batch_workspace_bytes(ps) -> int:
    arr = (swe_params * len(ps))(*ps)
    n = C.c_size_t(0)
    check(lib().swe_batch_workspace_bytes(arr, len(ps), C.byref(n)), "swe_batch_workspace_bytes")
    return n.value


def swe_batch_create(ps, bs, workspace: int, nbytes: int, stream: int) -> int:
    pa = (swe_params * len(ps))(*ps)
    ba = (swe_buffers * len(bs))(*bs)
    out = C.c_void_p(0)
    check(lib().swe_batch_create(pa, ba, len(ps), C.c_void_p(workspace), nbytes,
                                 C.c_void_p(stream), C.byref(out)), "swe_batch_create")
    return out.value


def swe_batch_destroy(b: int) -> None:
    check(lib().swe_batch_destroy(C.c_void_p(b)), "swe_batch_destroy")


def swe_batch_set_tiling(b: int, tx: int, ty: int) -> None:
    check(lib().swe_batch_set_tiling(C.c_void_p(b), tx, ty), "swe_batch_set_tiling")


def swe_batch_get_tiling(b: int):
    tx, ty, nt = C.c_int32(), C.c_int32(), C.c_int32()
    check(lib().swe_batch_get_tiling(C.c_void_p(b), C.byref(tx), C.byref(ty), C.byref(nt)),
          "swe_batch_get_tiling")
    return tx.value, ty.value, nt.value


def swe_batch_autotune(b: int, trial_steps: int):
    tx, ty, ms = C.c_int32(), C.c_int32(), C.c_double()
    check(lib().swe_batch_autotune(C.c_void_p(b), trial_steps, C.byref(tx), C.byref(ty),
                                   C.byref(ms)), "swe_batch_autotune")
    return tx.value, ty.value, ms.value


def swe_batch_set_rain(b: int, member: int, rain: float) -> None:
    check(lib().swe_batch_set_rain(C.c_void_p(b), member, rain), "swe_batch_set_rain")


def swe_batch_set_dt_log(b: int, member: int, ptr: int, capacity: int) -> None:
    check(lib().swe_batch_set_dt_log(C.c_void_p(b), member, C.c_void_p(ptr), capacity),
          "swe_batch_set_dt_log")


def swe_batch_step(b: int, nsteps: int, t_end: float = float("inf")) -> None:
    check(lib().swe_batch_step(C.c_void_p(b), nsteps, t_end), "swe_batch_step")


def swe_batch_get_time(b: int, member: int):
    t, dt, n = C.c_double(), C.c_double(), C.c_int64()
    check(lib().swe_batch_get_time(C.c_void_p(b), member, C.byref(t), C.byref(dt),
                                   C.byref(n)), "swe_batch_get_time")
    return t.value, dt.value, n.value


def swe_batch_get_status(b: int, count: int):
    flags = (C.c_uint32 * count)()
    rc = lib().swe_batch_get_status(C.c_void_p(b), flags, count)
    return rc, list(flags)


# -- adjoint ---------------------------------------------------------------------

def swe_adj_workspace_bytes(p, nsteps, ckpt_every, ngauges, every) -> int:
    n = C.c_size_t(0)
    check(lib().swe_adj_workspace_bytes(C.byref(p), nsteps, ckpt_every, ngauges, every,
                                        C.byref(n)), "swe_adj_workspace_bytes")
    return n.value


def swe_adj_create(p, b, nsteps, ckpt_every, gauges_ptr, ngauges, every, obs_ptr,
                   workspace, nbytes, stream) -> int:
    out = C.c_void_p(0)
    check(lib().swe_adj_create(C.byref(p), C.byref(b), nsteps, ckpt_every,
                               C.c_void_p(gauges_ptr), ngauges, every, C.c_void_p(obs_ptr),
                               C.c_void_p(workspace), nbytes, C.c_void_p(stream),
                               C.byref(out)), "swe_adj_create")
    return out.value


def swe_adj_destroy(a: int) -> None:
    check(lib().swe_adj_destroy(C.c_void_p(a)), "swe_adj_destroy")


def swe_adj_set_dts(a: int, ptr) -> None:
    check(lib().swe_adj_set_dts(C.c_void_p(a), C.c_void_p(ptr)), "swe_adj_set_dts")


def swe_adj_get_dts(a: int, ptr: int) -> None:
    check(lib().swe_adj_get_dts(C.c_void_p(a), C.c_void_p(ptr)), "swe_adj_get_dts")


def swe_adj_forward(a: int) -> float:
    loss = C.c_double(0.0)
    check(lib().swe_adj_forward(C.c_void_p(a), C.byref(loss)), "swe_adj_forward")
    return loss.value


def swe_adj_backward(a: int, grad_ptr: int) -> None:
    check(lib().swe_adj_backward(C.c_void_p(a), C.c_void_p(grad_ptr)), "swe_adj_backward")


def swe_adj_get_series(a: int, ptr: int) -> None:
    check(lib().swe_adj_get_series(C.c_void_p(a), C.c_void_p(ptr)), "swe_adj_get_series")


def swe_flow_dir_f32(z: int, nx: int, ny: int, code: int, rows: int, stream: int) -> None:
    check(lib().swe_flow_dir_f32(C.c_void_p(z), nx, ny, C.c_void_p(code), rows,
                                 C.c_void_p(stream)), "swe_flow_dir_f32")


def swe_flow_dir_f64(z: int, nx: int, ny: int, code: int, rows: int, stream: int) -> None:
    check(lib().swe_flow_dir_f64(C.c_void_p(z), nx, ny, C.c_void_p(code), rows,
                                 C.c_void_p(stream)), "swe_flow_dir_f64")


def swe_flow_dir_rows(nx: int, ny: int, elem_bytes: int) -> int:
    r = C.c_int32(0)
    check(lib().swe_flow_dir_rows(nx, ny, elem_bytes, C.byref(r)), "swe_flow_dir_rows")
    return r.value
