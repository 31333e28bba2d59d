"""Pins of the oracle's FD weights and Laplacian (Sec. IV.A, derivative expressions)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import laplacian, second_derivative_weights, weights_f64

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fd_weights.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        order, vals = line.split(":")
        out[int(order)] = [Fraction(v) for v in vals.split()]
    return out


@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_weights_match_published_values(order):
    # order 2 is the paper's printed example; 4-8 are Fornberg's table.
    assert second_derivative_weights(order) == _golden()[order]


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12, 14, 16])
def test_weights_match_closed_form(order):
    # Independent closed form: c_k = 2 (-1)^(k+1) (M!)^2 / (k^2 (M-k)! (M+k)!),
    # c_0 = -2 sum c_k.  The oracle solves the moment system instead.
    m = order // 2
    ck = [Fraction(2 * (-1) ** (k + 1) * math.factorial(m) ** 2,
                   k * k * math.factorial(m - k) * math.factorial(m + k)) for k in range(1, m + 1)]
    assert second_derivative_weights(order) == [-2 * sum(ck)] + ck


@pytest.mark.parametrize("order", [2, 4, 8, 14, 16])
def test_weights_accuracy_is_exactly_order(order):
    # Exact on x^j for j <= order+1 (2 on x^2, 0 otherwise); not exact on x^(order+2).
    c = second_derivative_weights(order)
    m = order // 2
    for j in range(order + 3):
        mom = sum(c[abs(k)] * Fraction(k) ** j for k in range(-m, m + 1))
        if j <= order + 1:
            assert mom == (2 if j == 2 else 0), (order, j)
        else:
            assert mom != 0


@pytest.mark.parametrize("order", [2, 4, 8, 16])
def test_weights_reject_bad_orders(order):
    for bad in (0, 1, 3, order + 1, -2):
        with pytest.raises(ValueError):
            second_derivative_weights(bad)


@pytest.mark.parametrize("order,ndim", [(4, 2), (8, 3), (16, 2)])
def test_laplacian_exact_on_polynomials(order, ndim):
    # Separable polynomial of degree order+1 per axis with anisotropic spacing:
    # the stencil must reproduce the analytic Laplacian at every point whose
    # stencil stays inside the array.
    rng = np.random.default_rng(11)
    m = order // 2
    n = [2 * m + 5 + a for a in range(ndim)]
    h = [0.7, 1.3, 0.9][:ndim]
    deg = order + 1
    coefs = [rng.standard_normal(deg + 1) * 0.1 ** np.arange(deg + 1) for _ in range(ndim)]
    grids = np.meshgrid(*[np.arange(n[a]) * h[a] - 0.5 * n[a] * h[a] for a in range(ndim)], indexing="ij")
    polys = [np.polynomial.Polynomial(c) for c in coefs]
    f = sum(polys[a](grids[a]) for a in range(ndim))
    exact = sum(polys[a].deriv(2)(grids[a]) for a in range(ndim))
    lap = laplacian(f, h, order)
    inner = tuple(slice(m, n[a] - m) for a in range(ndim))
    err = np.max(np.abs(lap[inner] - exact[inner])) / np.max(np.abs(exact[inner]))
    assert err < 1e-9
    # ...and one degree more is not reproduced (the order is not higher than stated).
    f2 = sum(np.polynomial.Polynomial(np.r_[np.zeros(deg + 1), 1.0])(grids[a]) for a in range(ndim))
    ex2 = sum(np.polynomial.Polynomial(np.r_[np.zeros(deg + 1), 1.0]).deriv(2)(grids[a]) for a in range(ndim))
    assert np.max(np.abs(laplacian(f2, h, order)[inner] - ex2[inner])) > 1e-6 * np.max(np.abs(ex2[inner]))


def test_laplacian_zero_outside_grid():
    # A single unit impulse at the corner: the Laplacian is the stencil itself,
    # truncated (values beyond the array are zero, nothing wraps around).
    order = 8
    c = weights_f64(order)
    u = np.zeros((12, 14))
    u[0, 0] = 1.0
    lap = laplacian(u, (1.0, 2.0), order)
    assert lap[0, 0] == pytest.approx(c[0] + c[0] / 4.0)
    for k in range(1, 5):
        assert lap[k, 0] == pytest.approx(c[k])
        assert lap[0, k] == pytest.approx(c[k] / 4.0)
    assert lap[-1, 0] == 0.0 and lap[0, -1] == 0.0 and lap[5, 0] == 0.0


def test_laplacian_periodic_symbol():
    # On a periodic grid, sin(xi j) is an eigenvector with eigenvalue
    # h^-2 (c_0 + 2 sum c_k cos(k xi)); compare with a brute-force dense matrix.
    order, n, h = 8, 24, 0.5
    c = weights_f64(order)
    m = order // 2
    mat = np.zeros((n, n))
    for i in range(n):
        for k in range(-m, m + 1):
            mat[i, (i + k) % n] += c[abs(k)] / h ** 2
    j = np.arange(n)
    for mode in (1, 3, 7, 12):
        xi = 2 * np.pi * mode / n
        f = np.sin(xi * j)
        assert np.allclose(laplacian(f, (h,), order, periodic=True), mat @ f, atol=1e-12)
