"""Torch-facing wrapper of the C ABI: tensors for device memory, the current
stream for ordering.  No arithmetic of the method happens here."""

from __future__ import annotations

import math
from typing import Optional

import numpy as np
import torch

from . import capi


def _dev(a, device) -> torch.Tensor:
    t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64))
    return t.to(device=device).contiguous()


def params_from(wl) -> capi.swe_params:
    return capi.make_params(**wl.params())


def _attach_fields(b: capi.swe_buffers, wl, device) -> dict:
    """Device copies of the workload's optional rain and soil fields, their
    pointers set in ``b``; the returned tensors must outlive the context."""
    out = {}
    for attr, field in (("rain_w", "rain_w"), ("ks_f", "ks"), ("psi_f", "psi"),
                        ("dtheta_f", "dtheta")):
        a = getattr(wl, attr)
        if a is not None:
            out[field] = _dev(a, device)
            setattr(b, field, out[field].data_ptr())
    return out


class Solver:
    """One simulation on one GPU.

    The state tensors ``h``, ``qx``, ``qy`` (and ``vinf`` with infiltration)
    are owned here and handed to the library by pointer; after ``step`` they
    hold the new state (stream-ordered).
    """

    def __init__(self, wl, device: str = "cuda", dt_log: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU")
        self.device = torch.device(device)
        self.params = params_from(wl)
        self.nx, self.ny = wl.nx, wl.ny
        self.h = _dev(wl.h, self.device)
        self.qx = _dev(wl.qx, self.device)
        self.qy = _dev(wl.qy, self.device)
        self.z = _dev(wl.z, self.device)
        self.fric = None if wl.fric is None else _dev(wl.fric, self.device)
        if wl.infil_on:
            v = np.zeros((wl.ny, wl.nx)) if wl.vinf is None else wl.vinf
            self.vinf = _dev(v, self.device)
        else:
            self.vinf = None
        nbytes = capi.swe_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        b = capi.swe_buffers()
        b.h, b.qx, b.qy = self.h.data_ptr(), self.qx.data_ptr(), self.qy.data_ptr()
        b.z = self.z.data_ptr()
        b.fric = self.fric.data_ptr() if self.fric is not None else None
        b.vinf = self.vinf.data_ptr() if self.vinf is not None else None
        self.fields = _attach_fields(b, wl, self.device)
        self._buffers = b
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = capi.swe_create(self.params, b, aligned, nbytes,
                                   self.stream.cuda_stream)
        if wl.rain_t is not None:
            capi.swe_set_hyetograph(self.ctx, wl.rain_t, wl.rain_r)
        self.dt_log = None
        if dt_log:
            self.dt_log = torch.zeros(dt_log, dtype=torch.float64, device=self.device)
            capi.swe_set_dt_log(self.ctx, self.dt_log.data_ptr(), dt_log)

    def close(self):
        if getattr(self, "ctx", None):
            capi.swe_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping ---------------------------------------------------------
    def step(self, nsteps: int, t_end: float = math.inf) -> None:
        capi.swe_step(self.ctx, nsteps, t_end)

    def set_tiling(self, tx: int, ty: int = 0) -> None:
        capi.swe_set_tiling(self.ctx, tx, ty)

    def tiling(self):
        return capi.swe_get_tiling(self.ctx)

    def profile_begin(self, max_steps: int) -> None:
        capi.swe_profile_begin(self.ctx, max_steps)

    def profile_end(self):
        """(ms in the rate kernel, ms in the update kernel, steps)."""
        return capi.swe_profile_end(self.ctx)

    def time(self):
        """(t, last_dt, steps); synchronizes."""
        return capi.swe_get_time(self.ctx)

    def status(self):
        return capi.swe_get_status(self.ctx)

    def set_time(self, t: float) -> None:
        capi.swe_set_time(self.ctx, t)

    def set_rain(self, r: float) -> None:
        capi.swe_set_rain(self.ctx, r)

    def set_hyetograph(self, t_pts, r) -> None:
        """Piecewise-constant rain r(t) (None removes it); synchronizes."""
        capi.swe_set_hyetograph(self.ctx, t_pts, r)

    def diagnostics(self) -> capi.swe_diag:
        return capi.swe_get_diagnostics(self.ctx)

    def rate(self, h: torch.Tensor, qx: torch.Tensor, qy: torch.Tensor):
        ph = torch.empty_like(h)
        pqx = torch.empty_like(h)
        pqy = torch.empty_like(h)
        amax = capi.swe_rate(self.ctx, h.data_ptr(), qx.data_ptr(), qy.data_ptr(),
                             ph.data_ptr(), pqx.data_ptr(), pqy.data_ptr())
        return ph, pqx, pqy, amax

    # -- state access -----------------------------------------------------
    def state(self):
        torch.cuda.synchronize(self.device)
        out = dict(h=self.h.cpu().numpy(), qx=self.qx.cpu().numpy(),
                   qy=self.qy.cpu().numpy())
        if self.vinf is not None:
            out["vinf"] = self.vinf.cpu().numpy()
        return out

    def set_state(self, h, qx, qy, vinf=None) -> None:
        self.h.copy_(torch.as_tensor(np.asarray(h, dtype=np.float64)))
        self.qx.copy_(torch.as_tensor(np.asarray(qx, dtype=np.float64)))
        self.qy.copy_(torch.as_tensor(np.asarray(qy, dtype=np.float64)))
        if vinf is not None and self.vinf is not None:
            self.vinf.copy_(torch.as_tensor(np.asarray(vinf, dtype=np.float64)))

    def set_boundary_values(self, side: int, h_b: float = 0.0, q_b: float = 0.0) -> None:
        """New imposed depth / inflow discharge of an imposed side (0 west,
        1 east, 2 south, 3 north) for the steps that follow."""
        capi.swe_set_boundary_values(self.ctx, side, h_b, q_b)

    def set_gauges(self, cells, every: int, max_samples: int) -> None:
        """Record h at the flat cell indices `cells` after every `every`
        steps from now on (at most max_samples samples); empty cells stop
        recording."""
        cells = np.asarray(cells, dtype=np.int32).ravel()
        if cells.size == 0:
            capi.swe_set_gauges(self.ctx, 0, 0, 1, 0, 0)
            self._gauge_cells = self._gauge_series = None
            return
        self._gauge_cells = torch.from_numpy(cells.copy()).to(self.device)
        self._gauge_series = torch.full((max_samples, cells.size), math.nan,
                                        dtype=torch.float64, device=self.device)
        capi.swe_set_gauges(self.ctx, self._gauge_cells.data_ptr(), cells.size, every,
                            self._gauge_series.data_ptr(), max_samples)

    def gauges(self) -> np.ndarray:
        """The samples recorded so far, one row of gauge depths each."""
        if getattr(self, "_gauge_series", None) is None:
            return np.zeros((0, 0))
        out = np.empty(tuple(self._gauge_series.shape), dtype=np.float64)
        n = capi.swe_get_gauges(self.ctx, out)
        return out[:n]

    def dts(self, n: Optional[int] = None) -> np.ndarray:
        if self.dt_log is None:
            raise RuntimeError("no dt log")
        _, _, steps = self.time()
        k = steps if n is None else n
        return self.dt_log[:k].cpu().numpy()


class Ensemble:
    """Independent simulations of uneven sizes stepped together on one GPU
    (one launch per stage for the whole ensemble, one block per tile)."""

    def __init__(self, workloads, device: str = "cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU")
        self.device = torch.device(device)
        self.count = len(workloads)
        self.params = [params_from(wl) for wl in workloads]
        self.members = []
        bufs = []
        for wl in workloads:
            m = {"h": _dev(wl.h, self.device), "qx": _dev(wl.qx, self.device),
                 "qy": _dev(wl.qy, self.device), "z": _dev(wl.z, self.device),
                 "fric": None if wl.fric is None else _dev(wl.fric, self.device),
                 "vinf": None}
            if wl.infil_on:
                v = np.zeros((wl.ny, wl.nx)) if wl.vinf is None else wl.vinf
                m["vinf"] = _dev(v, self.device)
            b = capi.swe_buffers()
            b.h, b.qx, b.qy = m["h"].data_ptr(), m["qx"].data_ptr(), m["qy"].data_ptr()
            b.z = m["z"].data_ptr()
            b.fric = m["fric"].data_ptr() if m["fric"] is not None else None
            b.vinf = m["vinf"].data_ptr() if m["vinf"] is not None else None
            m["fields"] = _attach_fields(b, wl, self.device)
            self.members.append(m)
            bufs.append(b)
        self._bufs = bufs
        nbytes = capi.swe_batch_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        self.stream = torch.cuda.current_stream(self.device)
        self.handle = capi.swe_batch_create(self.params, bufs, aligned, nbytes,
                                            self.stream.cuda_stream)
        for k, wl in enumerate(workloads):
            if wl.rain_t is not None:
                capi.swe_batch_set_hyetograph(self.handle, k, wl.rain_t, wl.rain_r)
        self.cells = sum(int(p.nx) * int(p.ny) for p in self.params)

    def close(self):
        if getattr(self, "handle", None):
            capi.swe_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, nsteps: int, t_end: float = math.inf) -> None:
        capi.swe_batch_step(self.handle, nsteps, t_end)

    def set_tiling(self, tx: int, ty: int) -> None:
        capi.swe_batch_set_tiling(self.handle, tx, ty)

    def tiling(self):
        return capi.swe_batch_get_tiling(self.handle)

    def autotune(self, trial_steps: int = 8):
        """(tx, ty, ms per step) of the fastest tile shape; state untouched."""
        return capi.swe_batch_autotune(self.handle, trial_steps)

    def set_rain(self, member: int, rain: float) -> None:
        capi.swe_batch_set_rain(self.handle, member, rain)

    def set_boundary_values(self, member: int, side: int, h_b: float = 0.0,
                            q_b: float = 0.0) -> None:
        capi.swe_batch_set_boundary_values(self.handle, member, side, h_b, q_b)

    def set_hyetograph(self, member: int, t_pts, r) -> None:
        capi.swe_batch_set_hyetograph(self.handle, member, t_pts, r)

    def time(self, member: int):
        return capi.swe_batch_get_time(self.handle, member)

    def status(self):
        return capi.swe_batch_get_status(self.handle, self.count)

    def state(self, member: int):
        torch.cuda.synchronize(self.device)
        m = self.members[member]
        out = {k: m[k].cpu().numpy() for k in ("h", "qx", "qy")}
        if m["vinf"] is not None:
            out["vinf"] = m["vinf"].cpu().numpy()
        return out


class Calibration:
    """Gauge-misfit loss of a run and its adjoint gradient with respect to the
    friction field (swe_adj_*).  The friction field lives in ``self.fric``
    (device); ``forward`` runs the simulation, ``backward`` returns dL/dfric
    of the last forward pass.  Each forward pass chooses its time steps by
    eq. (cfl) for the current field (the gradient is taken with them frozen)
    unless ``set_dts`` fixed them."""

    def __init__(self, wl, gauges, every: int, obs, nsteps: int, ckpt_every: int = 0,
                 device: str = "cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU")
        if wl.fric is None:
            raise ValueError("the workload needs a friction field")
        if any(getattr(wl, a) is not None for a in ("rain_t", "rain_w", "ks_f", "psi_f",
                                                    "dtheta_f")):
            raise ValueError("the adjoint takes uniform, constant rain and no soil fields")
        self.device = torch.device(device)
        self.params = params_from(wl)
        self.nx, self.ny = wl.nx, wl.ny
        self.nsteps = nsteps
        self.every = every
        self.h = _dev(wl.h, self.device)
        self.qx = _dev(wl.qx, self.device)
        self.qy = _dev(wl.qy, self.device)
        self.z = _dev(wl.z, self.device)
        self.fric = _dev(wl.fric, self.device)
        self.gauges = torch.as_tensor(np.ascontiguousarray(gauges, dtype=np.int32)).to(self.device)
        self.obs = _dev(np.asarray(obs, dtype=np.float64).reshape(-1), self.device)
        ng = int(self.gauges.numel())
        assert self.obs.numel() == (nsteps // every) * ng
        ck = ckpt_every or max(1, int(round(math.sqrt(nsteps))))
        nbytes = capi.swe_adj_workspace_bytes(self.params, nsteps, ck, ng, every)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        b = capi.swe_buffers()
        b.h, b.qx, b.qy = self.h.data_ptr(), self.qx.data_ptr(), self.qy.data_ptr()
        b.z = self.z.data_ptr()
        b.fric = self.fric.data_ptr()
        b.vinf = None
        self._b = b
        self.stream = torch.cuda.current_stream(self.device)
        self.handle = capi.swe_adj_create(self.params, b, nsteps, ck, self.gauges.data_ptr(), ng,
                                          every, self.obs.data_ptr(), aligned, nbytes,
                                          self.stream.cuda_stream)
        self.ckpt_every = ck
        self.fixed_dts = False
        # number of forward passes so far: a backward pass belongs to the last
        self.generation = 0

    def close(self):
        if getattr(self, "handle", None):
            capi.swe_adj_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_dts(self, dts) -> None:
        """Fix the time steps of every later forward pass to ``dts``
        (nsteps values); None returns to eq. (cfl) steps per forward pass."""
        if dts is None:
            capi.swe_adj_set_dts(self.handle, None)
            self.fixed_dts = False
            return
        t = _dev(np.asarray(dts, dtype=np.float64), self.device)
        capi.swe_adj_set_dts(self.handle, t.data_ptr())
        torch.cuda.synchronize(self.device)
        self.fixed_dts = True

    def dts(self) -> np.ndarray:
        t = torch.empty(self.nsteps, dtype=torch.float64, device=self.device)
        capi.swe_adj_get_dts(self.handle, t.data_ptr())
        torch.cuda.synchronize(self.device)
        return t.cpu().numpy()

    def forward(self) -> float:
        if not self.fixed_dts:
            # the library freezes the steps a pass chose; the next field
            # chooses its own
            capi.swe_adj_set_dts(self.handle, None)
        loss = capi.swe_adj_forward(self.handle)
        self.generation += 1
        return loss

    def series(self) -> np.ndarray:
        """Gauge depths of the last forward pass, one row per `every` steps."""
        rows = self.nsteps // self.every
        t = torch.empty(rows * int(self.gauges.numel()), dtype=torch.float64,
                        device=self.device)
        capi.swe_adj_get_series(self.handle, t.data_ptr())
        torch.cuda.synchronize(self.device)
        return t.cpu().numpy().reshape(rows, -1)

    def backward(self) -> torch.Tensor:
        g = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
        capi.swe_adj_backward(self.handle, g.data_ptr())
        return g


class GaugeMisfit(torch.autograd.Function):
    """loss = GaugeMisfit.apply(fric, calibration): the gauge-misfit loss of
    the calibration run as a differentiable function of the friction field
    (a float64 tensor on the GPU); the backward pass is the hand-written
    adjoint of the step."""

    @staticmethod
    def forward(ctx, fric: torch.Tensor, calib: "Calibration"):
        with torch.no_grad():
            calib.fric.copy_(fric.detach().to(calib.fric.dtype).reshape(calib.fric.shape))
        loss = calib.forward()
        ctx.calib = calib
        ctx.generation = calib.generation
        return torch.tensor(loss, dtype=torch.float64, device=fric.device)

    @staticmethod
    def backward(ctx, grad_out):
        if ctx.calib.generation != ctx.generation:
            raise RuntimeError("GaugeMisfit: the calibration ran another forward pass after "
                               "this loss; call backward on a loss before the next apply")
        g = ctx.calib.backward()
        return grad_out * g, None


def flow_directions(z: torch.Tensor, out: Optional[torch.Tensor] = None,
                    rows: int = 0) -> torch.Tensor:
    """Eight-neighbour flow-direction codes (0..8, uint8) of a [ny][nx]
    float32 or float64 DEM on the GPU (Section 5.2), enqueued on the current
    stream.  ``out`` may be given (uint8, same shape, contiguous)."""
    if z.dim() != 2 or not z.is_cuda or z.dtype not in (torch.float32, torch.float64):
        raise ValueError("z must be a 2-D float32 or float64 CUDA tensor")
    z = z.contiguous()
    ny, nx = z.shape
    if out is None:
        out = torch.empty((ny, nx), dtype=torch.uint8, device=z.device)
    elif out.shape != z.shape or out.dtype != torch.uint8 or not out.is_contiguous() \
            or out.device != z.device:
        raise ValueError("out must be a contiguous uint8 tensor shaped like z on its device")
    stream = torch.cuda.current_stream(z.device).cuda_stream
    fn = capi.swe_flow_dir_f32 if z.dtype == torch.float32 else capi.swe_flow_dir_f64
    with torch.cuda.device(z.device):
        fn(z.data_ptr(), nx, ny, out.data_ptr(), rows, stream)
    return out
