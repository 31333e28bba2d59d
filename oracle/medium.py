"""Model padding, absorbing-layer damping, update coefficients and the
stability limit, in FP64.

Test infrastructure: part of the plain CPU oracle (see ``oracle/__init__``).

Readings of the paper used here (the paper leaves them open):

* The computational grid is the physical model with ``nbl`` absorbing points
  added on every side (Sec. V.D: 201x201x70 plus 40 points per side gives
  281x281x150).  Inside the layer the squared slowness m is the value of the
  nearest physical edge cell (edge replication).
* Listing 1 adds ``damp * u.dt`` to ``m u_tt - laplace(u)`` with a spatially
  varying absorption field ``damp`` (Sec. V.C) but does not give its profile.
  Here damp = eta = sum over axes of eta_a(i_a), with
  eta_a = eta_max,a (d_a / nbl)^k, d_a the distance in points into the layer
  (0 in the physical region, nbl at the outer edge), and
  eta_max,a = (k+1) ln(1/R) / (v_ref nbl h_a).  For m u_tt + eta u_t a wave of
  speed v decays at rate eta v^2 / 2; the chosen eta_max makes the round trip
  through a layer of thickness nbl h_a attenuate by the factor R when
  v = v_ref.  v_ref is a fixed number, so eta does not depend on m.
* ``u.dt`` is the central difference (u[n+1] - u[n-1]) / (2 dt); solving
  m (u[n+1] - 2u[n] + u[n-1])/dt^2 + eta (u[n+1] - u[n-1])/(2 dt) = L u + q
  for u[n+1] (``solve(eqn, u.forward)`` of Listing 1) gives
  u[n+1] = A u[n] - B u[n-1] + C (L u[n] + q) with D+- = m +- eta dt / 2,
  A = 2 m / D+, B = D- / D+, C = dt^2 / D+.
* Stability: with eta = 0 the leapfrog scheme is stable when
  (v dt)^2 lambda_max <= 4, lambda_max being the largest eigenvalue of -L.
  The symbol of the order-P stencil peaks at the Nyquist wavenumber, where it
  equals sum_{k=-M..M} |c_k| / h^2 per axis, so
  dt_max = 2 / (v_max sqrt(sum_a sum_k |c_k| / h_a^2)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .fd import weights_f64

__all__ = ["pad_model", "fold_padding", "damping", "Coefficients", "coefficients", "dt_max"]


def pad_model(m: np.ndarray, nbl: int) -> np.ndarray:
    """Edge-replicate the physical model by ``nbl`` cells on every side."""
    return np.pad(np.asarray(m, dtype=np.float64), nbl, mode="edge")


def fold_padding(g_pad: np.ndarray, nbl: int) -> np.ndarray:
    """Adjoint of :func:`pad_model`: every padded cell's value is added onto
    the physical cell it was copied from."""
    g = np.asarray(g_pad, dtype=np.float64)
    for a in range(g.ndim):
        g = np.moveaxis(g, a, 0)
        n = g.shape[0] - 2 * nbl
        out = g[nbl:nbl + n].copy()
        out[0] += g[:nbl].sum(axis=0)
        out[-1] += g[nbl + n:].sum(axis=0)
        g = np.moveaxis(out, 0, a)
    return g


def damping(shape, nbl: int, spacing, power: int, reflection: float, vref: float) -> np.ndarray:
    """The absorption field eta on the padded grid (zero when nbl == 0)."""
    padded = tuple(int(n) + 2 * nbl for n in shape)
    eta = np.zeros(padded, dtype=np.float64)
    if nbl == 0:
        return eta
    for a, n in enumerate(shape):
        i = np.arange(n + 2 * nbl)
        depth = np.maximum(np.maximum(nbl - i, i - (n + nbl - 1)), 0).astype(np.float64)
        eta_max = (power + 1) * math.log(1.0 / reflection) / (vref * nbl * float(spacing[a]))
        prof = eta_max * (depth / nbl) ** power
        view = [1] * len(shape)
        view[a] = padded[a]
        eta = eta + prof.reshape(view)
    return eta


@dataclass
class Coefficients:
    A: np.ndarray
    B: np.ndarray
    C: np.ndarray


def coefficients(m_pad: np.ndarray, eta: np.ndarray, dt: float) -> Coefficients:
    """A, B, C of the explicit update for m u_tt + eta u_t - L u = q."""
    m_pad = np.asarray(m_pad, dtype=np.float64)
    d_plus = m_pad + eta * (dt / 2.0)
    d_minus = m_pad - eta * (dt / 2.0)
    return Coefficients(A=2.0 * m_pad / d_plus, B=d_minus / d_plus, C=dt * dt / d_plus)


def dt_max(order: int, spacing, vmax: float) -> float:
    """Largest stable time step of the undamped scheme for speeds <= vmax."""
    c = weights_f64(order)
    s = abs(c[0]) + 2.0 * float(np.sum(np.abs(c[1:])))
    return 2.0 / (vmax * math.sqrt(sum(s / float(h) ** 2 for h in spacing)))
