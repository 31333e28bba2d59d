"""Central finite-difference weights and the discrete Laplacian, in exact
rationals and FP64.

Test infrastructure: part of the plain CPU oracle.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark use it.

The paper (Sec. IV.A, "Derivative expressions") sets the accuracy of the
second derivative by one parameter, ``space_order``, and prints the order-2
case: f.dx2 = (f(x-h) - 2 f(x) + f(x+h)) / h^2.  For a general even order
P = 2M the symmetric (2M+1)-point stencil is *defined* here as the one that
differentiates every polynomial of degree <= 2M exactly.  With the symmetry
c_{-k} = c_k the odd moments vanish by themselves, so the weights solve the
M+1 even-moment equations

    sum_{k=-M..M} c_|k| k^j = 2 [j == 2],   j = 0, 2, ..., 2M,

which this module solves by exact Gaussian elimination over the rationals.
The Laplacian (Sec. IV.A, derivative expressions, the ``laplace`` shorthand; the 3-D form printed
as ``f.dx2 + f.dy2 + f.dz`` is read as ``... + f.dz2``) is the sum of the
per-axis second derivatives, with the field taken as zero outside the array
(the untouched outer halo of the generated code in Listing 3).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

__all__ = ["second_derivative_weights", "weights_f64", "laplacian"]


def _solve_exact(a: list[list[Fraction]], b: list[Fraction]) -> list[Fraction]:
    """Gauss-Jordan elimination over the rationals (no rounding anywhere)."""
    n = len(b)
    rows = [list(a[i]) + [b[i]] for i in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if rows[r][col] != 0)
        rows[col], rows[piv] = rows[piv], rows[col]
        p = rows[col][col]
        rows[col] = [v / p for v in rows[col]]
        for r in range(n):
            if r != col and rows[r][col] != 0:
                f = rows[r][col]
                rows[r] = [vr - f * vc for vr, vc in zip(rows[r], rows[col])]
    return [rows[i][n] for i in range(n)]


def second_derivative_weights(order: int) -> list[Fraction]:
    """Exact weights [c_0, c_1, ..., c_M] of the order-``order`` central
    second derivative (unit spacing).  ``order`` must be even and >= 2."""
    if not isinstance(order, (int, np.integer)) or order < 2 or order % 2:
        raise ValueError(f"space order must be an even integer >= 2, got {order!r}")
    m = order // 2
    # Unknowns c_0..c_M; equation for moment j = 2e, e = 0..M:
    #   c_0 [j == 0] + 2 sum_{k>=1} c_k k^j = 2 [j == 2]
    a, b = [], []
    for e in range(m + 1):
        j = 2 * e
        row = [Fraction(1 if j == 0 else 0)]
        row += [Fraction(2 * k**j) for k in range(1, m + 1)]
        a.append(row)
        b.append(Fraction(2 if j == 2 else 0))
    return _solve_exact(a, b)


def weights_f64(order: int) -> np.ndarray:
    """The exact weights rounded once to FP64, as an array [c_0..c_M]."""
    return np.array([float(c) for c in second_derivative_weights(order)], dtype=np.float64)


def laplacian(u: np.ndarray, spacing, order: int, periodic: bool = False) -> np.ndarray:
    """L_P u[i] = sum_a h_a^-2 sum_{k=-M..M} c_|k| u[i + k e_a].

    ``u`` is an FP64 array of any dimension; axis a has spacing ``spacing[a]``.
    Outside the array u is zero (``periodic=False``) or wraps around
    (``periodic=True``; a test-only option used for closed-form dispersion
    checks, needs every axis length >= M).
    """
    u = np.asarray(u, dtype=np.float64)
    c = weights_f64(order)
    m = order // 2
    if periodic and min(u.shape) < m:
        raise ValueError("periodic Laplacian needs every axis length >= M")
    ext = np.pad(u, m, mode="wrap" if periodic else "constant")
    out = np.zeros_like(u)
    for a in range(u.ndim):
        inv_h2 = 1.0 / float(spacing[a]) ** 2
        for k in range(-m, m + 1):
            sl = [slice(m, m + n) for n in u.shape]
            sl[a] = slice(m + k, m + k + u.shape[a])
            out += (c[abs(k)] * inv_h2) * ext[tuple(sl)]
    return out
