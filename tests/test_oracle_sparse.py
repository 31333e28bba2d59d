"""Pins of the oracle's off-grid interpolation and injection."""
import numpy as np
import pytest

from oracle import interpolation, sample, spread


@pytest.mark.parametrize("ndim", [2, 3])
def test_weights_sum_to_one_and_linear_fields_are_exact(ndim):
    rng = np.random.default_rng(ndim)
    shape_phys = (9, 11, 7)[:ndim]
    nbl = 3
    h = (2.0, 3.0, 5.0)[:ndim]
    padded = tuple(n + 2 * nbl for n in shape_phys)
    lo = np.array([-nbl * h[a] for a in range(ndim)])
    hi = np.array([(shape_phys[a] - 1 + nbl) * h[a] for a in range(ndim)])
    pts = lo + rng.random((50, ndim)) * (hi - lo)
    nodes, w = interpolation(pts, h, nbl, padded)
    assert nodes.shape == (50, 2 ** ndim, ndim)
    assert np.allclose(w.sum(axis=1), 1.0, atol=1e-14)
    assert np.all(w >= 0)
    # an affine field a0 + sum_a a_a x_a is reproduced exactly
    coef = rng.standard_normal(ndim + 1)
    grids = np.meshgrid(*[(np.arange(padded[a]) - nbl) * h[a] for a in range(ndim)], indexing="ij")
    f = coef[0] + sum(coef[a + 1] * grids[a] for a in range(ndim))
    exact = coef[0] + pts @ coef[1:]
    assert np.allclose(sample(f, nodes, w), exact, rtol=1e-13, atol=1e-12)


def test_on_grid_point_hits_one_node():
    nodes, w = interpolation([[20.0, 30.0]], (10.0, 10.0), 2, (10, 10))
    j = np.argmax(w[0])
    assert w[0, j] == 1.0 and tuple(nodes[0, j]) == (4, 5)


def test_point_on_last_plane_is_valid():
    # padded axis of 10 points with nbl = 1: x = 80 m is s = 9, the last node;
    # it is valid and takes i0 = 8 with weight 1 on node 9.
    nodes, w = interpolation([[80.0, 0.0]], (10.0, 10.0), 1, (10, 10))
    j = np.argmax(w[0])
    assert w[0, j] == 1.0 and nodes[0, j, 0] == 9 and nodes[0].max() <= 9


@pytest.mark.parametrize("bad", [[[-25.0, 0.0]], [[0.0, 105.0]], [[np.nan, 0.0]]])
def test_outside_points_are_rejected(bad):
    with pytest.raises(ValueError):
        interpolation(bad, (10.0, 10.0), 2, (12, 13))


def test_spread_is_the_transpose_of_sample():
    rng = np.random.default_rng(5)
    padded = (14, 12, 10)
    pts = rng.random((40, 3)) * np.array([10.0, 8.0, 6.0])
    nodes, w = interpolation(pts, (1.0, 1.0, 1.0), 2, padded)
    f = rng.standard_normal(padded)
    vals = rng.standard_normal(40)
    lhs = np.dot(sample(f, nodes, w), vals)
    rhs = np.sum(f * spread(padded, nodes, w, vals))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
