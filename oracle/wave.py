"""The acoustic operator: forward modelling, its adjoint, the FWI misfit and
the adjoint-state gradient, in FP64 NumPy.

Test infrastructure: part of the plain CPU oracle (see ``oracle/__init__``).

What is computed (Sec. V.A, Eqs. 1-4, with the damping of Listing 1; the
coefficient readings are stated in ``oracle.medium``):

forward, Eq. (1) with ``damp * u.dt`` and zero initial state:
    u[-1] = u[0] = 0
    u[n+1] = A u[n] - B u[n-1] + C (L u[n] + S q[n]),   n = 0 .. nt-2
    d[n]   = R u[n]                                      n = 0 .. nt-1
  q[n] is the wavelet sampled at t = n dt, S the source injection (transposed
  interpolation over the cell volume), R the receiver interpolation.  The
  receivers record after the step that injected q[n], so d[0] = R u[0] = 0.

misfit, Eq. (2): Phi = 1/2 || d - d_obs ||^2 (plain sum, no quadrature weights).

adjoint, Eq. (4) run backwards in time (Listing 2: the damping term flips
sign and the stencil is solved for ``v.backward``; with the central u.dt this
is the forward kernel time-reversed):
    mu[nt] = mu[nt+1] = 0
    mu[n] = A mu[n+1] - B mu[n+2] + C (L mu[n+1] + R^T y[n]),  n = nt-1 .. 0
  and the adjoint of the source map, F^T y:  s[n] = S^T mu[n+1] for
  n <= nt-2, s[nt-1] = 0.

gradient, Eq. (3) (adjoint-state), as the exact derivative of the discrete
misfit with respect to the padded m, driven by y = d - d_obs:
    g = -(1/dt^2) sum_{n=1..nt-1} u[n] * (mu[n] - 2 mu[n+1] + mu[n+2])
  The paper writes the sum of u v_tt without the sign; differentiating the
  discrete scheme gives the minus sign above, which the finite-difference
  and Taylor tests of Sec. V.B (Eqs. 7-8) confirm.  The gradient with
  respect to the physical model folds the padding (``medium.fold_padding``).

Eq. (3) needs u at every time step ("full storage of the forward wavefield").
``gradient(..., checkpoint_every=K)`` instead keeps the pair
(u[jK], u[jK-1]) every K steps and recomputes each segment during the reverse
sweep; the arithmetic is the same, so the result is bitwise equal.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .fd import laplacian
from .medium import coefficients, damping, dt_max, fold_padding, pad_model
from .sparse import cell_volume, interpolation, sample, spread

__all__ = ["Problem", "Operator", "misfit"]


@dataclass
class Problem:
    """Everything that defines one shot except the model and the wavelet."""
    shape: tuple                 # physical points per axis, axis 0 = depth
    spacing: tuple               # metres per axis
    order: int                   # even space order P
    nbl: int                     # absorbing points added on every side
    dt: float                    # seconds
    nt: int                      # time samples (nt-1 steps)
    src_coords: np.ndarray       # [nsrc, ndim] metres from the physical origin
    rec_coords: np.ndarray       # [nrec, ndim]
    damp_power: int = 1
    damp_R: float = 1e-3
    damp_vref: float = 1500.0
    periodic: bool = False       # test-only: wrap-around Laplacian, no damping
    padded_shape: tuple = field(init=False)

    def __post_init__(self):
        self.shape = tuple(int(n) for n in self.shape)
        self.spacing = tuple(float(h) for h in self.spacing)
        self.padded_shape = tuple(n + 2 * self.nbl for n in self.shape)
        self.src_coords = np.atleast_2d(np.asarray(self.src_coords, dtype=np.float64)).reshape(-1, len(self.shape))
        self.rec_coords = np.atleast_2d(np.asarray(self.rec_coords, dtype=np.float64)).reshape(-1, len(self.shape))


class Operator:
    """The discrete forward/adjoint pair for one model."""

    def __init__(self, problem: Problem, m: np.ndarray, check_cfl: bool = True, backend: str = "numpy"):
        p = problem
        self.p = p
        if backend not in ("numpy", "c") or (backend == "c" and p.periodic):
            raise ValueError("backend is 'numpy' or 'c' (the C step has no periodic option)")
        self.backend = backend
        m = np.asarray(m, dtype=np.float64)
        if m.shape != p.shape:
            raise ValueError(f"model shape {m.shape} != problem shape {p.shape}")
        if not np.all(np.isfinite(m)) or np.any(m <= 0):
            raise ValueError("squared slowness must be finite and positive")
        if check_cfl and p.dt > dt_max(p.order, p.spacing, float(np.sqrt(1.0 / m.min()))):
            raise ValueError("dt exceeds the stability limit")
        self.m_pad = pad_model(m, p.nbl)
        if p.periodic:
            self.eta = np.zeros(p.padded_shape)
        else:
            self.eta = damping(p.shape, p.nbl, p.spacing, p.damp_power, p.damp_R, p.damp_vref)
        k = coefficients(self.m_pad, self.eta, p.dt)
        self.A, self.B, self.C = k.A, k.B, k.C
        self.src = interpolation(p.src_coords, p.spacing, p.nbl, p.padded_shape) if len(p.src_coords) else None
        self.rec = interpolation(p.rec_coords, p.spacing, p.nbl, p.padded_shape) if len(p.rec_coords) else None
        self.vol = cell_volume(p.spacing)

    # -- one step of the recurrence -------------------------------------------
    def _lap(self, u):
        return laplacian(u, self.p.spacing, self.p.order, periodic=self.p.periodic)

    def step(self, u, u_prev, q_n=None):
        """u[n+1] from u[n], u[n-1] and the wavelet sample q[n] (one per source)."""
        if self.backend == "c":
            extra = None
            if self.src is not None and q_n is not None:
                extra = spread(self.p.padded_shape, *self.src, q_n)
            return self._cstep(u, u_prev, extra, self.vol)
        rhs = self._lap(u)
        if self.src is not None and q_n is not None:
            rhs = rhs + spread(self.p.padded_shape, *self.src, q_n) / self.vol
        return self.A * u - self.B * u_prev + self.C * rhs

    def adjoint_step(self, mu1, mu2, y_n=None):
        """mu[n] from mu[n+1], mu[n+2] and the receiver samples y[n]."""
        if self.backend == "c":
            extra = None
            if self.rec is not None and y_n is not None:
                extra = spread(self.p.padded_shape, *self.rec, y_n)
            return self._cstep(mu1, mu2, extra, 1.0)
        rhs = self._lap(mu1)
        if self.rec is not None and y_n is not None:
            rhs = rhs + spread(self.p.padded_shape, *self.rec, y_n)
        return self.A * mu1 - self.B * mu2 + self.C * rhs

    def _cstep(self, u, up, extra, div):
        from . import cref
        from .fd import weights_f64
        if not hasattr(self, "_w"):
            self._w = weights_f64(self.p.order)
            self.A, self.B, self.C = (np.ascontiguousarray(x) for x in (self.A, self.B, self.C))
        return cref.step(u, up, self.A, self.B, self.C, extra, div, self.p.spacing, self._w)

    def record(self, u):
        if self.rec is None:
            return np.zeros(0)
        return sample(u, *self.rec)

    # -- forward ---------------------------------------------------------------
    def forward(self, wavelet, state=None, keep=False, checkpoint_every=None):
        """Run nt-1 steps.

        wavelet: [nt, nsrc] (or [nt] for one source).
        state:   optional (u[0], u[-1]) to start from instead of zeros.
        Returns a dict with ``traces`` [nt, nrec], ``u`` = u[nt-1],
        ``u_prev`` = u[nt-2], and on request ``history`` (all u[n]) or
        ``checkpoints`` {j: (u[jK], u[jK-1])}.
        """
        p = self.p
        q = _as_2d(wavelet, p.nt)
        shape = p.padded_shape
        if state is None:
            u, u_prev = np.zeros(shape), np.zeros(shape)
        else:
            u, u_prev = (np.array(s, dtype=np.float64) for s in state)
        nrec = 0 if self.rec is None else self.rec[0].shape[0]
        traces = np.zeros((p.nt, nrec))
        traces[0] = self.record(u)
        history = [u] if keep else None
        ckpts = {} if checkpoint_every else None
        for n in range(p.nt):
            if ckpts is not None and n % checkpoint_every == 0:
                ckpts[n // checkpoint_every] = (u, u_prev)
            if n == p.nt - 1:
                break
            u_next = self.step(u, u_prev, q[n] if q.shape[1] else None)
            u_prev, u = u, u_next
            traces[n + 1] = self.record(u)
            if keep:
                history.append(u)
        out = {"traces": traces, "u": u, "u_prev": u_prev}
        if keep:
            out["history"] = history
        if ckpts is not None:
            out["checkpoints"] = ckpts
        return out

    def _recompute_segment(self, q, ckpts, K, j):
        """u[jK .. min(jK+K, nt)-1] from the stored pair (u[jK], u[jK-1])."""
        u, u_prev = ckpts[j]
        seg = [u]
        for n in range(j * K, min(j * K + K, self.p.nt) - 1):
            u_next = self.step(u, u_prev, q[n] if q.shape[1] else None)
            u_prev, u = u, u_next
            seg.append(u)
        return seg

    # -- adjoint ---------------------------------------------------------------
    def adjoint(self, y, history=None, wavelet=None, checkpoints=None, checkpoint_every=None):
        """Adjoint sweep driven by receiver data y [nt, nrec].

        Returns a dict with ``src_adj`` = F^T y [nt, nsrc] and ``mu0`` = mu[0].
        When the forward wavefield is supplied (``history``, or ``wavelet`` +
        ``checkpoints`` + ``checkpoint_every``) it also returns ``grad_pad``,
        the gradient with respect to the padded m.
        """
        p = self.p
        y = _as_2d(y, p.nt)
        shape = p.padded_shape
        nsrc = 0 if self.src is None else self.src[0].shape[0]
        src_adj = np.zeros((p.nt, nsrc))
        imaging = history is not None or checkpoints is not None
        if checkpoints is not None:
            q = _as_2d(wavelet, p.nt)
            K = checkpoint_every
        g = np.zeros(shape) if imaging else None
        mu1, mu2 = np.zeros(shape), np.zeros(shape)
        seg, seg_j = None, None
        for n in range(p.nt - 1, -1, -1):
            if nsrc and n <= p.nt - 2:
                src_adj[n] = sample(mu1, *self.src) / self.vol
            mu = self.adjoint_step(mu1, mu2, y[n] if y.shape[1] else None)
            if imaging and n >= 1:
                if history is not None:
                    u_n = history[n]
                else:
                    j = n // K
                    if seg_j != j:
                        seg, seg_j = self._recompute_segment(q, checkpoints, K, j), j
                    u_n = seg[n - j * K]
                g += u_n * (mu - 2.0 * mu1 + mu2)
            mu2, mu1 = mu1, mu
        out = {"src_adj": src_adj, "mu0": mu1}
        if imaging:
            out["grad_pad"] = -g / (p.dt * p.dt)
        return out

    # -- Born (linearised) modelling --------------------------------------------
    def born(self, wavelet, dm):
        """J dm: the derivative of the traces with respect to the physical
        model in the direction dm (the linear map whose adjoint is the
        gradient of Eq. 3).  Differentiating the discrete scheme with eta fixed:
            du[-1] = du[0] = 0,
            du[n+1] = A du[n] - B du[n-1] + C L du[n]
                      - (C / dt^2) dm_pad * (u[n+1] - 2 u[n] + u[n-1]),
            dd[n] = R du[n],
        with dm_pad the edge-replicated dm (the padding is linear in m).
        Returns the traces [nt, nrec] of du."""
        p = self.p
        q = _as_2d(wavelet, p.nt)
        dm_pad = pad_model(np.asarray(dm, dtype=np.float64), p.nbl)
        shape = p.padded_shape
        u, u_prev = np.zeros(shape), np.zeros(shape)
        du, du_prev = np.zeros(shape), np.zeros(shape)
        nrec = 0 if self.rec is None else self.rec[0].shape[0]
        traces = np.zeros((p.nt, nrec))
        for n in range(p.nt - 1):
            u_next = self.step(u, u_prev, q[n] if q.shape[1] else None)
            born_src = -(self.C / (p.dt * p.dt)) * dm_pad * (u_next - 2.0 * u + u_prev)
            du_next = self.A * du - self.B * du_prev + self.C * self._lap(du) + born_src
            u_prev, u = u, u_next
            du_prev, du = du, du_next
            traces[n + 1] = self.record(du)
        return traces

    # -- FWI gradient ----------------------------------------------------------
    def gradient(self, wavelet, d_obs, checkpoint_every=None):
        """Misfit, physical and padded gradient, and the modelled traces."""
        if checkpoint_every:
            fwd = self.forward(wavelet, checkpoint_every=checkpoint_every)
        else:
            fwd = self.forward(wavelet, keep=True)
        resid = fwd["traces"] - np.asarray(d_obs, dtype=np.float64)
        phi = misfit(fwd["traces"], d_obs)
        if checkpoint_every:
            adj = self.adjoint(resid, wavelet=wavelet, checkpoints=fwd["checkpoints"],
                               checkpoint_every=checkpoint_every)
        else:
            adj = self.adjoint(resid, history=fwd["history"])
        g_pad = adj["grad_pad"]
        return {"phi": phi, "grad": fold_padding(g_pad, self.p.nbl), "grad_pad": g_pad,
                "traces": fwd["traces"], "src_adj": adj["src_adj"]}


def misfit(traces, d_obs) -> float:
    """Eq. (2): half the squared L2 norm of the data residual."""
    r = np.asarray(traces, dtype=np.float64) - np.asarray(d_obs, dtype=np.float64)
    return 0.5 * float(np.sum(r * r))


def _as_2d(a, nt):
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    if a.shape[0] != nt:
        raise ValueError(f"time axis has {a.shape[0]} samples, expected {nt}")
    return a
