"""The adjoint with the imaging condition (Eq. 3, Sec. V.A) at the full size of
the order-16 gradient workload (400^3 + 40-point layer = 480^3 computed), in
the launch shapes its plans take: the autotuned one and, forced, the
two-wavefront 128 x 16 and 128 x 8 tiles and the built-in 64 x 8 tile.

The oracle cannot run 480^3 grids, so the shot is built to be checked on
sub-blocks: a few sources and receivers sit within 5 points of each of eight
sample points (grid corners, the absorbing layer, z-chunk, tile-row and
wavefront seams of every forced shape), far enough apart that over the
9 samples nothing travels from one group to another.  Each group's 145^3 block
is then an exact oracle problem of its own (helpers.oracle_block), and the
padded gradient, the traces and F^T of that group are compared with it on the
whole block."""
import numpy as np
import pytest

import oracle
import synth
from helpers import dev, gpu_plan, host, log, oracle_block, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu

NT = 9
R = 72            # block half-width: fields spread at most 8 (NT - 1) + 5 < R points from a group's centre
# z: multiples of 28 and 84 (chunk seams); y: multiples of 8 and 16 (tile rows);
# x: multiples of 64 and 128 (wavefront and tile seams); corners and edges in the layer
PTS = [(0, 0, 0), (479, 479, 479), (168, 16, 256), (336, 176, 128), (84, 336, 447), (252, 479, 64),
       (420, 96, 320), (240, 300, 300)]


def _groups(rng, shot):
    """Coordinates (metres from the physical origin) of 3 sources and 4
    receivers per sample point, within 5 points of it and inside the padded grid."""
    h = np.asarray(shot.spacing)
    P = np.array([n + 2 * shot.nbl for n in shot.shape])
    src, rec = [], []
    for p in PTS:
        p = np.asarray(p, dtype=np.float64)
        for out, k in ((src, 3), (rec, 4)):
            off = rng.uniform(-5.0, 5.0, size=(k, 3))
            g = np.clip(p + off, 0.0, P - 1.0)
            out.extend((g - shot.nbl) * h)
    return np.array(src), np.array(rec)


def test_full_size_order16_imaging_against_oracle_blocks(monkeypatch):
    import paper_1608_08658_amd as awe
    shot = synth.config_3d_gradient(nt=NT, nrec_side=2)
    rng = np.random.default_rng(71)
    shot.src_coords, shot.rec_coords = _groups(rng, shot)
    P = tuple(n + 2 * shot.nbl for n in shot.shape)
    M = shot.order // 2
    assert 8 * (NT - 1) + 5 < R and M == 8
    for i, a in enumerate(PTS):                      # no group reaches another's block
        for b in PTS[i + 1:]:
            assert max(abs(x - y) for x, y in zip(a, b)) > R + 8 * (NT - 1) + 5
    vmax = float(np.sqrt(1.0 / shot.m.min()))
    dt = 0.5 * oracle.dt_max(shot.order, shot.spacing, vmax)
    nsrc, nrec = len(shot.src_coords), len(shot.rec_coords)
    w = rng.standard_normal((NT, nsrc)).astype(np.float32)
    y = rng.standard_normal((NT, nrec)).astype(np.float32)

    results = {}
    for tile in (None, "5,84", "4,28", "1,28"):
        if tile is None:
            monkeypatch.delenv("AWE_TILE", raising=False)
        else:
            monkeypatch.setenv("AWE_TILE", tile)
        log(f"case order-16 imaging {P}, launch shape {tile or 'autotuned'}")
        plan = gpu_plan(shot, dt)
        plan.set_model(dev(shot.m))
        tr = plan.forward(dev(w), ckpt_every=2)
        sa, _ = plan.adjoint(dev(y), want_src_adj=True, want_grad=True)
        info = plan.info()
        results[tile] = (host(tr), host(sa), host(plan.gradient_padded()), info)
        plan.close()
        log(f"  shapes forward {info['forward_shape']}, imaging {info['imaging_shape']}")
    monkeypatch.delenv("AWE_TILE", raising=False)
    # every launch shape gives the same bits
    ref_key = "1,28"
    for key, (tr, sa, gp, _) in results.items():
        assert np.array_equal(tr, results[ref_key][0]), key
        assert np.array_equal(sa, results[ref_key][1]), key
        assert np.array_equal(gp, results[ref_key][2]), key
    tr, sa, gp, _ = results["5,84"]

    op = oracle.Operator(oracle_problem(shot, dt, nt=NT), shot.m, backend="c")
    for p in PTS:
        lo = [max(0, p[a] - R) for a in range(3)]
        hi = [min(P[a], p[a] + R + 1) for a in range(3)]
        sub, si, ri = oracle_block(op, lo, hi, backend="c")
        assert len(si) == 3 and len(ri) == 4, p
        fwd = sub.forward(w[:, si].astype(np.float64), keep=True)
        adj = sub.adjoint(y[:, ri].astype(np.float64), history=fwd["history"])
        sl = tuple(slice(lo[a], hi[a]) for a in range(3))
        g_blk = gp[sl]
        e_g = rel_l2(g_blk, adj["grad_pad"])
        e_tr = rel_l2(tr[:, ri], fwd["traces"])
        e_sa = rel_l2(sa[:, si], adj["src_adj"])
        nz = int(np.count_nonzero(adj["grad_pad"]))
        log(f"  block at {p}: gradient rel {e_g:.2e} ({nz} non-zero points), traces {e_tr:.2e}, F^T {e_sa:.2e}")
        assert nz > 1000
        assert e_g <= 1e-4 and e_tr <= 1e-4 and e_sa <= 1e-4, p
    # outside the blocks the gradient is zero
    mask = np.ones(P, dtype=bool)
    for p in PTS:
        mask[tuple(slice(max(0, p[a] - R), min(P[a], p[a] + R + 1)) for a in range(3))] = False
    assert not np.any(gp[mask])
