"""Pins of the oracle's padding, damping and stability limit."""
import math

import numpy as np
import pytest

import synth
from oracle import Operator, Problem, damping, dt_max, fold_padding, pad_model
from oracle.analytic import greens_2d


def test_padding_and_fold_are_adjoint():
    rng = np.random.default_rng(3)
    for shape, nbl in (((7, 9), 3), ((5, 6, 4), 2), ((4, 4), 0)):
        x = rng.standard_normal(shape)
        y = rng.standard_normal(tuple(n + 2 * nbl for n in shape))
        lhs = np.sum(pad_model(x, nbl) * y)
        rhs = np.sum(x * fold_padding(y, nbl))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_padding_replicates_edges():
    x = np.arange(12.0).reshape(3, 4)
    p = pad_model(x, 2)
    assert p.shape == (7, 8)
    assert np.all(p[:2, 2:6] == x[0]) and np.all(p[-2:, 2:6] == x[-1])
    assert np.all(p[2:5, :2] == x[:, :1]) and p[0, 0] == x[0, 0] and p[-1, -1] == x[-1, -1]


def test_damping_zero_inside_and_largest_at_edges():
    eta = damping((20, 30), 6, (10.0, 5.0), 2, 1e-3, 2000.0)
    assert eta.shape == (32, 42)
    assert np.all(eta[6:26, 6:36] == 0.0)
    assert np.all(eta >= 0.0)
    # the outer corner carries the sum of both axes' maxima
    assert eta[0, 0] == pytest.approx(eta[0, 20] + eta[16, 0])
    # monotone into the layer along each axis
    assert np.all(np.diff(eta[:7, 20]) < 0) and np.all(np.diff(eta[25:, 20]) > 0)


@pytest.mark.parametrize("order", [2, 4, 8, 16])
def test_dt_max_is_the_stability_boundary(order):
    # Undamped, periodic, constant velocity, rough random start: bounded just
    # below dt_max, exponential growth just above it.
    rng = np.random.default_rng(order)
    shape, h, v = (24, 30), (7.0, 11.0), 2000.0
    dtm = dt_max(order, h, v)
    u0 = rng.standard_normal(shape)
    peak = {}
    for f in (0.99, 1.01):
        p = Problem(shape, h, order, 0, f * dtm, 400, np.zeros((0, 2)), np.zeros((0, 2)), periodic=True)
        op = Operator(p, np.full(shape, 1.0 / v ** 2), check_cfl=False)
        out = op.forward(np.zeros((400, 0)), state=(u0, u0))
        peak[f] = np.max(np.abs(out["u"]))
    assert peak[0.99] < 50.0
    assert peak[1.01] > 1e6


def test_damping_layer_absorbs():
    # Boundary-reflected energy at a receiver near the top edge, with and
    # without the absorbing layer, against a much larger domain where nothing
    # comes back inside the window.  A missing or sign-flipped damping term
    # fails this.
    h, v, order, f0 = 10.0, 1500.0, 4, 10.0
    dt = 0.5 * dt_max(order, (h, h), v)
    nt = 420
    def run(n, nbl, off):
        shape = (n, n)
        src = [[off + 30 * h, off + 40 * h]]
        rec = [[off + 5 * h, off + 40 * h]]
        p = Problem(shape, (h, h), order, nbl, dt, nt, src, rec, damp_power=2, damp_vref=v)
        op = Operator(p, np.full(shape, 1.0 / v ** 2))
        return op.forward(synth.ricker(f0, dt, nt))["traces"][:, 0]
    big = run(300, 0, 110 * h)          # reflections arrive after the window
    undamped = run(81, 0, 0.0)
    damped = run(81, 30, 0.0)
    err_undamped = np.linalg.norm(undamped - big) / np.linalg.norm(big)
    err_damped = np.linalg.norm(damped - big) / np.linalg.norm(big)
    assert err_undamped > 0.3
    assert err_damped < 0.05


def test_greens_2d_quadrature_against_direct_integral():
    # The sigma-substituted quadrature equals the direct convolution integral.
    from scipy.integrate import quad
    s = synth.ricker_fn(10.0)
    r, v, t = 300.0, 1500.0, 0.35
    # 1/sqrt(v^2 tau^2 - r^2) = (tau - r/v)^(-1/2) / sqrt(v (v tau + r)): let
    # QUADPACK's algebraic-endpoint weight take the singular factor.
    direct = quad(lambda tau: s(t - tau) / math.sqrt(v * (v * tau + r)), r / v, t,
                  weight="alg", wvar=(-0.5, 0.0))[0] * v / (2 * math.pi)
    assert greens_2d(r, np.array([t]), v, s)[0] == pytest.approx(direct, rel=1e-6)
