"""Analytic solutions of Eq. (1) in a homogeneous, unbounded medium.

Test infrastructure: used only to pin the oracle to physics.

For m u_tt - laplace(u) = delta(x) s(t) with m = 1/v^2 and zero initial
state the solution is the source signature convolved with the free-space
Green's function:

* 3-D: u(r, t) = s(t - r/v) / (4 pi r).
* 2-D: u(r, t) = (v / 2 pi) int_{r/v}^{t} s(t - tau) / sqrt(v^2 tau^2 - r^2) dtau.
  With tau = r/v + sigma^2 the integrable singularity disappears:
  u(r, t) = (v / pi) int_0^{sqrt(t - r/v)} s(t - r/v - sigma^2) / sqrt(2 r v + v^2 sigma^2) dsigma.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["greens_3d", "greens_2d"]


def greens_3d(r: float, t: np.ndarray, v: float, signature) -> np.ndarray:
    t = np.asarray(t, dtype=np.float64)
    return np.asarray(signature(t - r / v), dtype=np.float64) / (4.0 * math.pi * r)


def greens_2d(r: float, t: np.ndarray, v: float, signature, nodes: int = 400) -> np.ndarray:
    """Gauss-Legendre quadrature in sigma over [0, sqrt(t - r/v)] for every t."""
    t = np.asarray(t, dtype=np.float64)
    x, w = np.polynomial.legendre.leggauss(nodes)
    out = np.zeros_like(t)
    for i, ti in enumerate(t):
        tail = ti - r / v
        if tail <= 0:
            continue
        top = math.sqrt(tail)
        sig = 0.5 * top * (x + 1.0)
        f = np.asarray(signature(tail - sig * sig), dtype=np.float64) / np.sqrt(2.0 * r * v + v * v * sig * sig)
        out[i] = (v / math.pi) * 0.5 * top * np.dot(w, f)
    return out
