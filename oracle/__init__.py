"""CPU oracle for the 2D shallow-water step (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The numerics live in
``oracle/swe_oracle.cpp`` (plain FP64 loops written from the paper); this
module compiles it with g++ and marshals numpy arrays through ctypes.  It
imports nothing from the HIP library package.
"""

from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "swe_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-shared", "-fPIC"]


def build(force: bool = False) -> str:
    """Compile the oracle library with g++ (always when ``force``)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", *CFLAGS, _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class OrcParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double),
                ("g", C.c_double), ("cfl", C.c_double),
                ("dt_max", C.c_double), ("h_eps", C.c_double),
                ("bc", C.c_int32 * 4), ("fric_law", C.c_int32),
                ("fric_coef", C.c_double), ("rain", C.c_double),
                ("infil_on", C.c_int32), ("ks", C.c_double),
                ("psi", C.c_double), ("dtheta", C.c_double),
                ("rain_n", C.c_int32), ("rain_t", C.POINTER(C.c_double)),
                ("rain_r", C.POINTER(C.c_double)), ("rain_w", C.POINTER(C.c_double)),
                ("ks_f", C.POINTER(C.c_double)), ("psi_f", C.POINTER(C.c_double)),
                ("dtheta_f", C.POINTER(C.c_double)), ("order", C.c_int32),
                ("flux", C.c_int32), ("bc_h", C.c_double * 4), ("bc_q", C.c_double * 4),
                ("dt_min", C.c_double), ("recon", C.c_int32)]


_lib = None


def lib(path: Optional[str] = None):
    """The oracle library (SWE_ORACLE_LIB overrides the path; the mutation
    tests use it to load deliberately broken builds)."""
    global _lib
    if _lib is None or path is not None:
        l = C.CDLL(path or os.environ.get("SWE_ORACLE_LIB") or build())
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        pp = C.POINTER(OrcParams)
        l.orc_rate.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp, dp]
        l.orc_stage.argtypes = [pp, dp, C.c_double, dp, dp, dp, dp, dp, dp, dp, dp]
        l.orc_time_step.argtypes = [pp, dp, C.c_double, C.c_double]
        l.orc_time_step.restype = C.c_double
        l.orc_run.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp, C.c_double,
                              C.c_int32, dp, ip]
        l.orc_step_fixed.argtypes = [pp, C.c_double, C.c_double, dp, dp, dp, dp, dp, dp]
        l.orc_minmod.argtypes = [C.c_double, C.c_double]
        l.orc_minmod.restype = C.c_double
        l.orc_num_threads.restype = C.c_int
        l.orc_set_num_threads.argtypes = [C.c_int]
        l.orc_muscl.argtypes = [dp, dp, dp, C.c_double, dp]
        l.orc_eno.argtypes = [dp, dp, dp, C.c_double, C.c_int, dp]
        l.orc_hll.argtypes = [C.c_double] + [C.c_double] * 6 + [dp]
        l.orc_face.argtypes = [C.c_double] + [C.c_double] * 8 + [dp, C.c_int32]
        l.orc_tangent_run.argtypes = [pp, dp, dp, dp, dp, dp, dp, C.c_int32, dp,
                                      ip, C.c_int32, C.c_int32, dp, dp, dp]
        l.orc_gauge_run.argtypes = [pp, dp, dp, dp, dp, dp, C.c_int32, dp, ip,
                                    C.c_int32, C.c_int32, dp]
        if path is not None:
            return l
        _lib = l
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def params(nx, ny, dx, dy, g=9.81, cfl=0.5, dt_max=math.inf, h_eps=1e-12,
           bc=(0, 0, 0, 0), fric_law=0, fric_coef=0.0, rain=0.0, infil_on=0,
           ks=0.0, psi=0.0, dtheta=0.0, order=2, flux=0, bc_h=(0.0,) * 4,
           bc_q=(0.0,) * 4, dt_min=0.0, recon=0) -> OrcParams:
    p = OrcParams()
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


_KEEP = "_arrays"


def params_of(wl) -> OrcParams:
    """Parameters of a workload, with its hyetograph and per-cell rain and
    Green-Ampt fields attached (the arrays are kept alive on the struct)."""
    p = params(**wl.params())
    keep = []

    def attach(name, a):
        if a is None:
            return
        a = _f64(a)
        keep.append(a)
        setattr(p, name, _dp(a))

    if wl.rain_t is not None:
        assert wl.rain_r is not None and len(wl.rain_t) == len(wl.rain_r)
        p.rain_n = len(wl.rain_t)
        attach("rain_t", wl.rain_t)
        attach("rain_r", wl.rain_r)
    attach("rain_w", wl.rain_w)
    attach("ks_f", wl.ks_f)
    attach("psi_f", wl.psi_f)
    attach("dtheta_f", wl.dtheta_f)
    setattr(p, _KEEP, keep)
    return p


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------
# Array-level API
# ----------------------------------------------------------------------------

def rate(p: OrcParams, h, qx, qy, z):
    """Phi(U) of one convective stage and the wave-speed bounds (Ax, Ay)."""
    h, qx, qy, z = map(_f64, (h, qx, qy, z))
    ph, pqx, pqy = (np.empty_like(h) for _ in range(3))
    amax = np.zeros(2)
    rc = lib().orc_rate(C.byref(p), _dp(h), _dp(qx), _dp(qy), _dp(z),
                        _dp(ph), _dp(pqx), _dp(pqy), _dp(amax))
    assert rc == 0
    return ph, pqx, pqy, amax


def stage(p: OrcParams, dt, h, qx, qy, z, fric=None):
    h, qx, qy, z = map(_f64, (h, qx, qy, z))
    fric = None if fric is None else _f64(fric)
    ho, qxo, qyo = (np.empty_like(h) for _ in range(3))
    amax = np.zeros(2)
    rc = lib().orc_stage(C.byref(p), _dp(fric), dt, _dp(h), _dp(qx), _dp(qy),
                         _dp(z), _dp(ho), _dp(qxo), _dp(qyo), _dp(amax))
    assert rc == 0
    return ho, qxo, qyo, amax


def time_step(p: OrcParams, amax, t, t_end) -> float:
    amax = _f64(amax)
    return lib().orc_time_step(C.byref(p), _dp(amax), t, t_end)


class State:
    """Mutable oracle state: h, qx, qy, vinf arrays plus the time."""

    def __init__(self, wl):
        self.p = params_of(wl)
        self.h = _f64(wl.h).copy()
        self.qx = _f64(wl.qx).copy()
        self.qy = _f64(wl.qy).copy()
        self.z = _f64(wl.z).copy()
        self.fric = None if wl.fric is None else _f64(wl.fric).copy()
        if wl.infil_on:
            self.vinf = (np.zeros_like(self.h) if wl.vinf is None
                         else _f64(wl.vinf).copy())
        else:
            self.vinf = None
        self.t = 0.0
        self.steps = 0
        self.dts = []

    def run(self, nsteps: int, t_end: float = math.inf) -> int:
        """Advance; returns the oracle status code (0 ok, 1 t_end reached)."""
        log = np.zeros(max(nsteps, 1))
        done = C.c_int32(0)
        t = C.c_double(self.t)
        rc = lib().orc_run(C.byref(self.p), _dp(self.h), _dp(self.qx),
                           _dp(self.qy), _dp(self.z), _dp(self.fric),
                           _dp(self.vinf), C.byref(t), t_end, nsteps,
                           _dp(log), C.byref(done))
        self.t = t.value
        self.steps += done.value
        self.dts.extend(log[:done.value].tolist())
        return rc

    def step_fixed(self, dt: float):
        rc = lib().orc_step_fixed(C.byref(self.p), self.t, dt, _dp(self.h),
                                  _dp(self.qx), _dp(self.qy), _dp(self.z),
                                  _dp(self.fric), _dp(self.vinf))
        assert rc == 0
        self.t += dt
        self.steps += 1


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (results are the
    same at any count)."""
    lib().orc_set_num_threads(int(n))


def minmod(a, b):
    return lib().orc_minmod(a, b)


def muscl(a, c, b, h_eps=1e-12):
    """prim triples {h, un, ut, eta} -> {h_m, h_p, z_m, z_p, un_m, un_p, ut_m, ut_p}."""
    a, c, b = (np.ascontiguousarray(x, dtype=np.float64) for x in (a, c, b))
    out = np.zeros(8)
    lib().orc_muscl(_dp(a), _dp(c), _dp(b), h_eps, _dp(out))
    return out


def eno(a, c, b, h_eps=1e-12, modified=False):
    """ENO (or modified ENO) face values of one cell, as muscl()."""
    a, c, b = (np.ascontiguousarray(x, dtype=np.float64) for x in (a, c, b))
    out = np.zeros(8)
    lib().orc_eno(_dp(a), _dp(c), _dp(b), h_eps, int(bool(modified)), _dp(out))
    return out


def hll(g, hL, unL, utL, hR, unR, utR):
    out = np.zeros(3)
    lib().orc_hll(g, hL, unL, utL, hR, unR, utR, _dp(out))
    return out


def face(g, hm, zm, unm, utm, hp, zp, unp, utp, flux=0):
    """{F0, F1, F2, sL, sR, speed} of one face (flux 0 HLL, 1 Rusanov,
    2 kinetic, 3 VFRoe-ncv)."""
    out = np.zeros(6)
    lib().orc_face(g, hm, zm, unm, utm, hp, zp, unp, utp, _dp(out), flux)
    return out


def tangent_run(p: OrcParams, h0, qx0, qy0, z, fric, dfric, dts, gauges,
                every, obs):
    """Loss and its derivative along dfric with the dt sequence frozen."""
    h0, qx0, qy0, z, fric = map(_f64, (h0, qx0, qy0, z, fric))
    dfric = _f64(dfric)
    dts = _f64(dts)
    gauges = np.ascontiguousarray(gauges, dtype=np.int32)
    obs = _f64(obs)
    loss, dloss = C.c_double(0.0), C.c_double(0.0)
    rc = lib().orc_tangent_run(C.byref(p), _dp(h0), _dp(qx0), _dp(qy0),
                               _dp(z), _dp(fric), _dp(dfric), len(dts),
                               _dp(dts), _ip(gauges), len(gauges), every,
                               _dp(obs), C.byref(loss), C.byref(dloss))
    assert rc == 0
    return loss.value, dloss.value


def gauge_run(p: OrcParams, h, qx, qy, z, fric, dts, gauges, every):
    h, qx, qy = (_f64(a).copy() for a in (h, qx, qy))
    z = _f64(z)
    fric = None if fric is None else _f64(fric)
    dts = _f64(dts)
    gauges = np.ascontiguousarray(gauges, dtype=np.int32)
    rows = len(dts) // every
    out = np.zeros((rows, len(gauges)))
    rc = lib().orc_gauge_run(C.byref(p), _dp(h), _dp(qx), _dp(qy), _dp(z),
                             _dp(fric), len(dts), _dp(dts), _ip(gauges),
                             len(gauges), every, _dp(out))
    assert rc == 0
    return out, (h, qx, qy)
