"""Blocked 2-D forward steps (several time steps per launch, the source
injected and the receivers sampled inside the launch; orders 2 and 4):
bit-identical to one step per launch (AWE_TB=0), with the source and
receivers on tile seams, step counts that leave a partial block, and chunked
stepping as the shot server drives it.  A blocked plan holds two more
fields, which shows that the blocked path was taken."""
import numpy as np
import pytest

import synth
from helpers import dev, gpu_plan, host, log, shot_dt, small_2d_shot

pytestmark = pytest.mark.gpu

TILE = 32


def _seam_shot(order, nt, seed):
    # padded grid 150 x 95 (nbl 10): tiles of 32 meet at padded indices 32, 64, ...
    shot = small_2d_shot(seed, order, shape=(130, 75), nbl=10, nt=nt, nrec=7)
    h = shot.spacing
    nbl = shot.nbl

    def phys(iz, ix, fz=0.0, fx=0.0):     # padded node index (+ fraction) -> physical coordinates
        return [(iz + fz - nbl) * h[0], (ix + fx - nbl) * h[1]]

    # a source whose four nodes straddle the seams in z and x
    shot.src_coords = np.array([phys(TILE - 1, TILE - 1, 0.4, 0.7)])
    shot.rec_coords = np.array([phys(TILE - 1, TILE - 1, 0.5, 0.5), phys(TILE, TILE, 0.2, 0.1),
                                phys(TILE - 1, 3, 0.9, 0.0), phys(2 * TILE - 1, 40, 0.3, 0.6),
                                phys(148, 93, 0.5, 0.5), phys(0, 0, 0.0, 0.0), phys(20, TILE - 1, 0.0, 0.99)])
    return shot


def _run(monkeypatch, shot, dt, blocked, chunks=None):
    monkeypatch.delenv("AWE_FUSE", raising=False)   # blocking needs the point operators in the launch
    if blocked:
        monkeypatch.delenv("AWE_TB", raising=False)
    else:
        monkeypatch.setenv("AWE_TB", "0")
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    w = dev(shot.wavelet(dt))
    import torch
    if chunks is None:
        tr = plan.forward(w)
    else:
        tr = torch.zeros((shot.nt, len(shot.rec_coords)), device="cuda")
        z = torch.zeros(plan.padded, device="cuda")
        plan.set_state(z, z)
        n = 0
        for c in chunks:
            plan.step(n, c, wavelet=w, traces=tr)
            n += c
    u, up = plan.get_state()
    out = (host(tr), host(u), host(up))
    held = plan.info()["bytes"]
    plan.close()
    return out, held


def _check(a, b, shot, what=""):
    (oa, held_a), (ob, held_b) = a, b
    field = 4 * np.prod([n + 2 * shot.nbl for n in shot.shape])
    assert held_a - held_b >= 2 * field, "the blocked path was not taken"
    for x, y, name in zip(oa, ob, ("traces", "u", "u_prev")):
        assert np.array_equal(x, y), (what, name)


@pytest.mark.parametrize("order", [2, 4])
def test_blocked_2d_forward_is_bitwise_equal_to_one_step_per_launch(monkeypatch, order):
    shot = _seam_shot(order, nt=23, seed=600 + order)
    dt = shot_dt(shot)
    a = _run(monkeypatch, shot, dt, blocked=True)
    b = _run(monkeypatch, shot, dt, blocked=False)
    log(f"order {order}: max |trace| {np.abs(b[0][0]).max():.3e}, max |u| {np.abs(b[0][1]).max():.3e}")
    assert np.abs(b[0][0]).max() > 0 and np.abs(b[0][1]).max() > 0
    _check(a, b, shot, order)


@pytest.mark.parametrize("order", [2, 4])
def test_blocked_2d_chunked_steps_are_bitwise_equal(monkeypatch, order):
    # the server's pattern: awe_step over chunks that do not align with the block length
    shot = _seam_shot(order, nt=40, seed=700 + order)
    dt = shot_dt(shot)
    chunks = [5, 1, 13, 3, 17]
    a = _run(monkeypatch, shot, dt, blocked=True, chunks=chunks)
    b = _run(monkeypatch, shot, dt, blocked=False, chunks=chunks)
    _check(a, b, shot, order)


def test_blocked_2d_large_grid_and_paper_small_case(monkeypatch):
    # many tiles (padded 700 x 1030, order 4) and the 121^2 order-4 small case
    rng = np.random.default_rng(5)
    shape = (660, 990)
    v = synth.layered_velocity(shape, rng, nlayers=(4, 7))
    shot = synth.Shot("tb-large", shape, (10.0, 10.0), 4, 20, 37, 1.0 / v ** 2,
                      np.array([[1000.3, 2000.7]]),
                      np.column_stack([np.full(300, 25.0), np.linspace(0, 9890.0, 300)]), 12.0,
                      damp_vref=float(v.min()))
    dt = shot_dt(shot)
    _check(_run(monkeypatch, shot, dt, blocked=True), _run(monkeypatch, shot, dt, blocked=False), shot, "large")
    small = synth.config_2d_small()
    dt = shot_dt(small)
    _check(_run(monkeypatch, small, dt, blocked=True), _run(monkeypatch, small, dt, blocked=False), small, "small")


@pytest.mark.parametrize("nt", [1, 2, 3, 5])
def test_blocked_2d_tiny_step_counts(monkeypatch, nt):
    # no step, one step (a launch of one), and partial blocks
    shot = _seam_shot(2, nt=nt, seed=800 + nt)
    dt = shot_dt(shot)
    _check(_run(monkeypatch, shot, dt, blocked=True), _run(monkeypatch, shot, dt, blocked=False), shot, nt)
