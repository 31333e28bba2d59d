"""Python front end of libawe: plans, the autograd Function and the shot server.

Torch is used for device memory and streams only; every step of the operator
runs in the library's HIP kernels.  Tensors passed in must be float32,
contiguous and on the current HIP device.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np

from . import _lib
from ._lib import AweError, Geometry, check, lib

__all__ = ["Plan", "Server", "Gradient", "make_geometry", "fd_weights", "dt_max", "footprint", "misfit",
           "sum_fields", "AweError"]


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, name, shape=None, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return C.c_void_p(t.data_ptr())


class GeometryHolder:
    """An awe_geometry plus the coordinate arrays it points into."""

    def __init__(self, shape, spacing, space_order, nbl, dt, nt, src_coords, rec_coords,
                 damp_power=1, damp_R=1e-3, damp_vref=1500.0):
        ndim = len(shape)
        self.src = np.ascontiguousarray(np.asarray(src_coords, dtype=np.float64).reshape(-1, ndim))
        self.rec = np.ascontiguousarray(np.asarray(rec_coords, dtype=np.float64).reshape(-1, ndim))
        g = Geometry()
        g.ndim = ndim
        g.space_order = int(space_order)
        for a in range(3):
            g.shape[a] = int(shape[a]) if a < ndim else 0
            g.spacing[a] = float(spacing[a]) if a < ndim else 0.0
        g.nbl = int(nbl)
        g.damp_power = int(damp_power)
        g.damp_R = float(damp_R)
        g.damp_vref = float(damp_vref)
        g.dt = float(dt)
        g.nt = int(nt)
        g.nsrc = self.src.shape[0]
        g.nrec = self.rec.shape[0]
        g.reserved = 0
        g.src_coords = self.src.ctypes.data_as(C.POINTER(C.c_double)) if g.nsrc else None
        g.rec_coords = self.rec.ctypes.data_as(C.POINTER(C.c_double)) if g.nrec else None
        self.g = g
        self.shape = tuple(int(n) for n in shape)
        self.padded = tuple(int(n) + 2 * int(nbl) for n in shape)


def make_geometry(**kw) -> GeometryHolder:
    return GeometryHolder(**kw)


def fd_weights(order: int) -> np.ndarray:
    out = (C.c_double * (order // 2 + 1))()
    check(lib().awe_fd_weights(order, out))
    return np.array(out[:])


def dt_max(ndim: int, order: int, spacing, vmax: float) -> float:
    h = (C.c_double * 3)(*[float(x) for x in spacing][:3], *([0.0] * (3 - len(spacing))))
    out = C.c_double()
    check(lib().awe_dt_max(ndim, order, h, float(vmax), C.byref(out)))
    return out.value


def footprint(geom: GeometryHolder, ckpt_every: int = 0, snapshots: int | None = None) -> int:
    """Device bytes of a plan: forward only, periodic checkpoints every
    ``ckpt_every`` steps, or (``snapshots`` given) binomial checkpointing."""
    out = C.c_uint64()
    if snapshots is not None:
        check(lib().awe_footprint_binomial(C.byref(geom.g), int(snapshots), C.byref(out)))
    else:
        check(lib().awe_footprint(C.byref(geom.g), int(ckpt_every), C.byref(out)))
    return out.value


def binomial_cost(nt: int, snapshots: int) -> tuple[int, int]:
    """(forward steps of a whole gradient, wavefield buffers held) for the
    binomial checkpointing schedule over nt samples with ``snapshots``
    stored states."""
    steps, fields = C.c_int64(), C.c_int32()
    check(lib().awe_binomial_cost(int(nt), int(snapshots), C.byref(steps), C.byref(fields)))
    return steps.value, fields.value


def sum_fields(parts, out=None):
    """Sum of equally shaped device tensors in list order, accumulated in FP64
    and rounded once (deterministic whatever order they were produced in)."""
    torch = _torch()
    if not parts:
        raise ValueError("no parts")
    if out is None:
        out = torch.empty_like(parts[0])
    ptrs = (C.c_void_p * len(parts))(*[_ptr(p, f"parts[{i}]", tuple(parts[0].shape)).value
                                       for i, p in enumerate(parts)])
    check(lib().awe_sum_fields(_ptr(out, "out", tuple(parts[0].shape)), ptrs, len(parts), parts[0].numel(),
                               _stream()))
    return out


def misfit(traces, d_obs, want_resid=True):
    """Phi = 1/2 ||traces - d_obs||^2 (FP64 sum on device) and the residual."""
    torch = _torch()
    n = traces.numel()
    resid = torch.empty_like(traces) if want_resid else None
    phi = C.c_double()
    check(lib().awe_misfit(_ptr(traces, "traces"), _ptr(d_obs, "d_obs", traces.shape), n,
                           _ptr(resid, "resid", allow_none=True), C.byref(phi), _stream()))
    return phi.value, resid


class Plan:
    """One modelling problem on the current device (wraps awe_plan)."""

    def __init__(self, shape, spacing, space_order, nbl, dt, nt, src_coords, rec_coords,
                 damp_power=1, damp_R=1e-3, damp_vref=1500.0):
        self.geom = GeometryHolder(shape, spacing, space_order, nbl, dt, nt, src_coords, rec_coords,
                                   damp_power, damp_R, damp_vref)
        g = self.geom.g
        self.ndim, self.nt, self.nsrc, self.nrec = g.ndim, g.nt, g.nsrc, g.nrec
        self.shape, self.padded = self.geom.shape, self.geom.padded
        self.dt = g.dt
        h = C.c_void_p()
        check(lib().awe_plan_create(C.byref(g), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan has been closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().awe_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        out = (C.c_int64 * 8)()
        check(lib().awe_plan_info(self.handle, out))
        return {"padded": tuple(out[:self.ndim]), "bytes": out[3], "forward_shape": (out[4], out[5]),
                "imaging_shape": (out[6], out[7])}

    def time_kernels(self, every=1):
        """Record HIP events around every ``every``-th step launch (0: off)."""
        check(lib().awe_plan_time_kernels(self.handle, int(every)))

    def kernel_times(self):
        """{kind: (launches timed, mean microseconds)} for 'step' (no imaging),
        'imaging' and 'points' (point operators launched on their own)."""
        out = (C.c_double * 6)()
        check(lib().awe_plan_kernel_times(self.handle, out))
        return {k: (int(out[2 * i]), out[2 * i + 1]) for i, k in enumerate(("step", "imaging", "points"))}

    def set_model(self, m):
        check(lib().awe_set_model(self.handle, _ptr(m, "m", self.shape), _stream()))

    def forward(self, wavelet, ckpt_every=0, traces=None, snapshots=None):
        """Traces of a forward run; ``ckpt_every`` > 0 keeps periodic
        checkpoints, ``snapshots`` (not None) the states of the binomial
        schedule, for a following gradient."""
        torch = _torch()
        if traces is None:
            traces = torch.empty((self.nt, self.nrec), dtype=torch.float32, device="cuda")
        w = _ptr(wavelet, "wavelet", (self.nt, self.nsrc), allow_none=self.nsrc == 0)
        tr = _ptr(traces, "traces", (self.nt, self.nrec))
        if snapshots is not None:
            check(lib().awe_forward_binomial(self.handle, w, tr, int(snapshots), _stream()))
        else:
            check(lib().awe_forward(self.handle, w, tr, int(ckpt_every), _stream()))
        return traces

    def forward_id(self):
        """Identifier of the forward state a gradient would read (changes with
        every set_model, forward and born, and when binomial states are used)."""
        out = C.c_int64()
        check(lib().awe_forward_id(self.handle, C.byref(out)))
        return out.value

    def adjoint(self, resid, want_src_adj=True, want_grad=False, forward_id=None):
        """F^T resid and, with ``want_grad``, the gradient.  ``forward_id``
        (from :meth:`forward_id` after the forward) makes the call fail with
        AWE_ESTATE if the plan no longer holds that forward."""
        torch = _torch()
        src_adj = torch.empty((self.nt, self.nsrc), dtype=torch.float32, device="cuda") if want_src_adj else None
        grad = torch.empty(self.shape, dtype=torch.float32, device="cuda") if want_grad else None
        args = (_ptr(resid, "resid", (self.nt, self.nrec)), _ptr(src_adj, "src_adj", allow_none=True),
                _ptr(grad, "grad", allow_none=True), _stream())
        if forward_id is None:
            check(lib().awe_adjoint(self.handle, *args))
        else:
            check(lib().awe_adjoint_checked(self.handle, int(forward_id), *args))
        return src_adj, grad

    def born(self, wavelet, dm, traces=None):
        """J dm: linearised traces for a model perturbation dm (physical shape)."""
        torch = _torch()
        if traces is None:
            traces = torch.empty((self.nt, self.nrec), dtype=torch.float32, device="cuda")
        check(lib().awe_born(self.handle, _ptr(wavelet, "wavelet", (self.nt, self.nsrc), allow_none=self.nsrc == 0),
                             _ptr(dm, "dm", self.shape), _ptr(traces, "traces", (self.nt, self.nrec)), _stream()))
        return traces

    def gradient_padded(self):
        torch = _torch()
        out = torch.empty(self.padded, dtype=torch.float32, device="cuda")
        check(lib().awe_get_gradient_padded(self.handle, _ptr(out, "g_pad"), _stream()))
        return out

    def set_state(self, u, u_prev):
        check(lib().awe_set_state(self.handle, _ptr(u, "u", self.padded), _ptr(u_prev, "u_prev", self.padded),
                                  _stream()))

    def step(self, n0, nsteps, wavelet=None, traces=None):
        check(lib().awe_step(self.handle, int(n0), int(nsteps),
                             _ptr(wavelet, "wavelet", (self.nt, self.nsrc), allow_none=True),
                             _ptr(traces, "traces", (self.nt, self.nrec), allow_none=True), _stream()))

    def step2_blocked(self, npairs, zchunk=0):
        """2 * npairs source-free steps, two per z-sweep (the temporal-blocking
        prototype; bit-identical to step, and slower)."""
        check(lib().awe_step2_blocked(self.handle, int(npairs), int(zchunk), _stream()))

    def get_state(self):
        torch = _torch()
        u = torch.empty(self.padded, dtype=torch.float32, device="cuda")
        up = torch.empty(self.padded, dtype=torch.float32, device="cuda")
        check(lib().awe_get_state(self.handle, _ptr(u, "u"), _ptr(up, "u_prev"), _stream()))
        return u, up


def _make_gradient_fn():
    torch = _torch()

    class Gradient(torch.autograd.Function):
        """traces = F(m, wavelet) on a plan; backward gives dL/dm (physical
        model, adjoint-state with checkpoints every ``ckpt_every`` steps, or
        with binomial checkpointing over ``snapshots`` stored states when
        that is given) and dL/dwavelet (F^T applied to dL/dtraces)."""

        @staticmethod
        def forward(ctx, m, wavelet, plan, ckpt_every=30, snapshots=None):
            plan.set_model(m.contiguous())
            need_m = ctx.needs_input_grad[0]
            if need_m and snapshots is not None:
                traces = plan.forward(wavelet.contiguous(), snapshots=snapshots)
            else:
                traces = plan.forward(wavelet.contiguous(), ckpt_every=ckpt_every if need_m else 0)
            ctx.plan = plan
            ctx.forward_id = plan.forward_id()
            return traces

        @staticmethod
        def backward(ctx, grad_traces):
            # the plan holds one forward state: a later forward on it makes
            # this backward fail (AWE_ESTATE) instead of differentiating that one
            plan = ctx.plan
            src_adj, grad = plan.adjoint(grad_traces.contiguous(), want_src_adj=ctx.needs_input_grad[1],
                                         want_grad=ctx.needs_input_grad[0], forward_id=ctx.forward_id)
            return grad, src_adj, None, None, None

    return Gradient


class _LazyGradient:
    _fn = None

    def __getattr__(self, name):
        if _LazyGradient._fn is None:
            _LazyGradient._fn = _make_gradient_fn()
        return getattr(_LazyGradient._fn, name)


Gradient = _LazyGradient()


class Server:
    """Shot server with continuous batching (wraps awe_server)."""

    def __init__(self, hbm_fraction=0.9, chunk_steps=64, max_active=16):
        h = C.c_void_p()
        check(lib().awe_server_create(float(hbm_fraction), int(chunk_steps), int(max_active), C.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, geom: GeometryHolder, m: np.ndarray, wavelet: np.ndarray):
        """Copies m [shape] and wavelet [nt, nsrc] (host, float32); returns (ticket, traces array)."""
        g = geom.g
        m = np.ascontiguousarray(m, dtype=np.float32)
        w = np.ascontiguousarray(wavelet, dtype=np.float32).reshape(g.nt, g.nsrc)
        traces = np.zeros((g.nt, g.nrec), dtype=np.float32)
        t = C.c_int64()
        check(lib().awe_server_submit(self._h, C.byref(g), C.c_void_p(m.ctypes.data), C.c_void_p(w.ctypes.data),
                                      C.c_void_p(traces.ctypes.data), C.byref(t)))
        self._keep[t.value] = (traces, geom)
        return t.value, traces

    def submit_gradient(self, geom: GeometryHolder, m: np.ndarray, wavelet: np.ndarray, d_obs: np.ndarray,
                        ckpt_every: int, grad, want_traces=True):
        """A gradient request: copies m, wavelet [nt, nsrc] and d_obs [nt, nrec]
        (host, float32); the gradient lands in ``grad`` (a device tensor of the
        physical shape, kept alive here until the request is done).  Returns
        (ticket, traces array or None, phi array of one value)."""
        g = geom.g
        m = np.ascontiguousarray(m, dtype=np.float32)
        w = np.ascontiguousarray(wavelet, dtype=np.float32).reshape(g.nt, g.nsrc)
        obs = np.ascontiguousarray(d_obs, dtype=np.float32).reshape(g.nt, g.nrec)
        traces = np.zeros((g.nt, g.nrec), dtype=np.float32) if want_traces else None
        phi = np.full(1, np.nan, dtype=np.float64)
        t = C.c_int64()
        check(lib().awe_server_submit_gradient(
            self._h, C.byref(g), C.c_void_p(m.ctypes.data), C.c_void_p(w.ctypes.data), C.c_void_p(obs.ctypes.data),
            int(ckpt_every), C.c_void_p(traces.ctypes.data) if traces is not None else None,
            _ptr(grad, "grad", geom.shape), phi.ctypes.data_as(C.POINTER(C.c_double)), C.byref(t)))
        self._keep[t.value] = (traces, phi, grad, geom)
        return t.value, traces, phi

    def poll(self, ticket):
        st = C.c_int32()
        times = (C.c_double * 4)()
        check(lib().awe_server_poll(self._h, int(ticket), C.byref(st), times))
        return st.value, tuple(times[:])

    def wait(self, ticket, timeout=600.0):
        check(lib().awe_server_wait(self._h, int(ticket), float(timeout)))

    def stats(self):
        out = (C.c_int64 * 8)()
        check(lib().awe_server_stats(self._h, out))
        keys = ("submitted", "admitted", "completed", "failed", "running", "queued", "bytes_reserved", "iterations")
        return dict(zip(keys, out[:]))

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().awe_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
