"""Off-grid point operators: receiver interpolation and its transpose,
source injection, in FP64.

Test infrastructure: part of the plain CPU oracle (see ``oracle/__init__``).

The paper calls out sparse-point interpolation for source insertion and
receiver sampling as the feature stencil languages lack (Sec. IV) without
naming the scheme; Listing 3 passes coordinates to the operator.  Reading
used here: multilinear interpolation on the padded grid, and injection is its
exact transpose divided by the cell volume prod_a h_a, so that the discrete
source integrates to the point source q = s(t) delta(x - x_s) of Eq. (1).

Coordinates are in metres from the first physical grid point, one column per
axis (axis 0 = depth).  On axis a: s = x_a / h_a + nbl, i0 = floor(s), and a
point exactly on the last grid plane uses i0 = n_a - 2 with weight 1 on the
far node.  A point outside [0, n_a - 1] in grid units is an error.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

__all__ = ["interpolation", "sample", "spread"]


def interpolation(coords, spacing, nbl: int, padded_shape):
    """Return (nodes [npts, 2^d, d] int64, weights [npts, 2^d] FP64)."""
    coords = np.atleast_2d(np.asarray(coords, dtype=np.float64))
    ndim = len(padded_shape)
    if coords.shape[1] != ndim:
        raise ValueError(f"coordinates need {ndim} columns, got {coords.shape[1]}")
    npts = coords.shape[0]
    i0 = np.zeros((npts, ndim), dtype=np.int64)
    frac = np.zeros((npts, ndim), dtype=np.float64)
    for a in range(ndim):
        s = coords[:, a] / float(spacing[a]) + nbl
        last = padded_shape[a] - 1
        if np.any(~np.isfinite(s)) or np.any(s < 0) or np.any(s > last):
            raise ValueError(f"a point lies outside the padded grid on axis {a}")
        base = np.minimum(np.floor(s).astype(np.int64), last - 1)
        i0[:, a] = base
        frac[:, a] = s - base
    corners = list(itertools.product((0, 1), repeat=ndim))
    nodes = np.zeros((npts, len(corners), ndim), dtype=np.int64)
    weights = np.ones((npts, len(corners)), dtype=np.float64)
    for j, bits in enumerate(corners):
        for a, b in enumerate(bits):
            nodes[:, j, a] = i0[:, a] + b
            weights[:, j] *= frac[:, a] if b else (1.0 - frac[:, a])
    return nodes, weights


def sample(field: np.ndarray, nodes: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """Interpolate ``field`` at every point: out[p] = sum_j w[p,j] field[node[p,j]]."""
    vals = field[tuple(nodes[..., a] for a in range(field.ndim))]
    return np.sum(weights * vals, axis=1)


def spread(shape, nodes: np.ndarray, weights: np.ndarray, values: np.ndarray) -> np.ndarray:
    """Transpose of :func:`sample`: a field holding sum_p w[p,j] values[p] at
    each node (duplicates accumulate)."""
    out = np.zeros(shape, dtype=np.float64)
    contrib = weights * np.asarray(values, dtype=np.float64)[:, None]
    np.add.at(out, tuple(nodes[..., a] for a in range(len(shape))), contrib)
    return out


def cell_volume(spacing) -> float:
    return math.prod(float(h) for h in spacing)
