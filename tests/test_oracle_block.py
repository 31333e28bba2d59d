"""The block-restricted oracle (helpers.oracle_block) used by the full-size
GPU checks: on a grid small enough for the whole oracle, a block holding a
group of sources and receivers, sized so that no field reaches its faces,
gives the same traces, F^T and padded gradient as the whole grid (the
gradient is zero outside the block).  A block too small for the run must
differ, so the check is not vacuous."""
import numpy as np

import oracle
from helpers import oracle_block


def _problem_and_fields(nt, seed=0):
    rng = np.random.default_rng(seed)
    shape, nbl, h, order = (44, 40, 48), 6, (10.0, 11.0, 9.0), 4
    P = np.array([n + 2 * nbl for n in shape])
    v = 1500.0 + 1000.0 * rng.random(shape)
    centre = np.array([20.0, 18.0, 25.0])
    src = (np.clip(centre + rng.uniform(-3, 3, (2, 3)), 0, P - 1) - nbl) * h
    rec = (np.clip(centre + rng.uniform(-3, 3, (3, 3)), 0, P - 1) - nbl) * h
    dt = 0.5 * oracle.dt_max(order, h, float(v.max()))
    prob = oracle.Problem(shape, h, order, nbl, dt, nt, src, rec, damp_power=2, damp_vref=1500.0)
    op = oracle.Operator(prob, 1.0 / v ** 2)
    w = rng.standard_normal((nt, 2))
    y = rng.standard_normal((nt, 3))
    return op, centre.astype(int), w, y


def _run(op, w, y):
    fwd = op.forward(w, keep=True)
    adj = op.adjoint(y, history=fwd["history"])
    return fwd["traces"], adj["src_adj"], adj["grad_pad"]


def test_block_equals_whole_grid():
    nt = 5
    op, c, w, y = _problem_and_fields(nt)
    tr, sa, gp = _run(op, w, y)
    r = 2 * (nt - 1) + 3 + 2                     # M = 2: fields spread 2 points per step
    lo = [c[a] - r for a in range(3)]
    hi = [c[a] + r + 1 for a in range(3)]
    sub, si, ri = oracle_block(op, lo, hi)
    assert list(si) == [0, 1] and list(ri) == [0, 1, 2]
    tr_b, sa_b, gp_b = _run(sub, w[:, si], y[:, ri])
    sl = tuple(slice(lo[a], hi[a]) for a in range(3))
    assert np.allclose(tr_b, tr, rtol=0, atol=1e-13 * np.abs(tr).max())
    assert np.allclose(sa_b, sa, rtol=0, atol=1e-13 * np.abs(sa).max())
    assert np.allclose(gp_b, gp[sl], rtol=0, atol=1e-13 * np.abs(gp).max())
    outside = np.ones(gp.shape, dtype=bool)
    outside[sl] = False
    assert not np.any(gp[outside])


def test_too_small_block_differs():
    # the tightest block holding every source and receiver node: all points
    # are kept, but the fields reach past its faces, so the result changes
    nt = 5
    op, c, w, y = _problem_and_fields(nt)
    _, _, gp = _run(op, w, y)
    nodes = np.concatenate([op.src[0].reshape(-1, 3), op.rec[0].reshape(-1, 3)])
    lo, hi = list(nodes.min(axis=0)), list(nodes.max(axis=0) + 1)
    sub, si, ri = oracle_block(op, lo, hi)
    assert len(si) == 2 and len(ri) == 3
    _, _, gp_b = _run(sub, w[:, si], y[:, ri])
    sl = tuple(slice(lo[a], hi[a]) for a in range(3))
    assert np.max(np.abs(gp_b - gp[sl])) > 1e-6 * np.abs(gp).max()
