"""The temporal-blocking prototype (two 3-D steps per z-sweep, no point
operators): bit for bit the state two single steps give, across tile and
z-chunk seams, ragged tails, orders 2-8, and at the full 336^3 size of the
forward workload; and its argument checks."""
import numpy as np
import pytest

import synth
from helpers import dev, gpu_plan, host, log, shot_dt, small_3d_shot

pytestmark = pytest.mark.gpu


def _pair(shot, npairs, zchunk, seed=7):
    dt = shot_dt(shot)
    rng = np.random.default_rng(seed)
    P = tuple(n + 2 * shot.nbl for n in shot.shape)
    u0 = synth.random_state(rng, P, 3.0).astype(np.float32)
    um = (u0 * 0.999).astype(np.float32)
    plan = gpu_plan(shot, dt, nt=2 * npairs + 1, src=np.zeros((0, 3)))
    plan.set_model(dev(shot.m))
    plan.set_state(dev(u0), dev(um))
    plan.step(0, 2 * npairs)
    ref = [host(a) for a in plan.get_state()]
    plan.set_state(dev(u0), dev(um))
    plan.step2_blocked(npairs, zchunk)
    got = [host(a) for a in plan.get_state()]
    # and single steps continue from the blocked state as from their own
    plan.step(0, 2)
    after = [host(a) for a in plan.get_state()]
    plan.set_state(dev(ref[0]), dev(ref[1]))
    plan.step(0, 2)
    after_ref = [host(a) for a in plan.get_state()]
    plan.close()
    return ref, got, after, after_ref


# grids spanning several owned tiles in x (64 - 2M columns each) and y
# (32 - 2M rows), several z chunks, ragged tails on every axis
@pytest.mark.parametrize("order,shape,npairs,zchunk", [
    (8, (40, 46, 150), 1, 0),
    (8, (37, 61, 121), 3, 9),
    (6, (33, 70, 130), 2, 16),
    (4, (30, 52, 141), 2, 7),
    (2, (21, 35, 129), 4, 5),
])
def test_two_steps_per_sweep_equal_two_single_steps(order, shape, npairs, zchunk):
    shot = small_3d_shot(1000 + order, order, shape=shape, nbl=5)
    log(f"case order {order} shape {shape} pairs {npairs} zchunk {zchunk}")
    ref, got, after, after_ref = _pair(shot, npairs, zchunk)
    for a, b, name in zip(got, ref, ("u", "u_prev")):
        assert np.array_equal(a, b), name
    assert np.abs(ref[0]).max() > 0
    for a, b, name in zip(after, after_ref, ("u", "u_prev")):
        assert np.array_equal(a, b), name


# chunks starting fewer than M planes into the grid compute level-1 planes at
# z < 0, whose LDS ring slots once aliased the staging planes other waves were
# reading (results then varied from run to run near tile seams); each case
# runs the blocked launch three times from one state
@pytest.mark.parametrize("order,zchunk", [(8, 3), (6, 2), (6, 16), (4, 1), (2, 5)])
def test_two_steps_per_sweep_repeatable_near_the_first_plane(order, zchunk):
    shot = small_3d_shot(1200 + order, order, shape=(24, 60, 125), nbl=4)
    log(f"case order {order} zchunk {zchunk}")
    dt = shot_dt(shot)
    rng = np.random.default_rng(11)
    P = tuple(n + 2 * shot.nbl for n in shot.shape)
    u0 = synth.random_state(rng, P, 3.0).astype(np.float32)
    um = (u0 * 0.999).astype(np.float32)
    plan = gpu_plan(shot, dt, nt=5, src=np.zeros((0, 3)))
    plan.set_model(dev(shot.m))
    plan.set_state(dev(u0), dev(um))
    plan.step(0, 4)
    ref = [host(a) for a in plan.get_state()]
    for rep in range(3):
        plan.set_state(dev(u0), dev(um))
        plan.step2_blocked(2, zchunk)
        got = [host(a) for a in plan.get_state()]
        for a, b, name in zip(got, ref, ("u", "u_prev")):
            assert np.array_equal(a, b), f"{name}, run {rep}: {int((a != b).sum())} points differ"
    plan.close()


def test_two_steps_per_sweep_full_size():
    # the 336^3 forward workload's grid (256^3 + 40-point layer), order 8
    shot = synth.config_3d_forward(nt=5)
    log("case 336^3 order 8")
    ref, got, _, _ = _pair(shot, 1, 0)
    for a, b, name in zip(got, ref, ("u", "u_prev")):
        assert np.array_equal(a, b), name


def test_two_steps_per_sweep_arguments():
    import paper_1608_08658_amd as awe
    shot = small_3d_shot(1100, 8, shape=(20, 22, 30), nbl=4, nt=10)
    dt = shot_dt(shot)
    plan = gpu_plan(shot, dt)                          # with a source
    plan.set_model(dev(shot.m))
    with pytest.raises(awe.AweError):
        plan.step2_blocked(1)
    plan.close()
    shot16 = small_3d_shot(1101, 16, shape=(20, 22, 30), nbl=4, nt=10)
    plan = gpu_plan(shot16, shot_dt(shot16), src=np.zeros((0, 3)))
    plan.set_model(dev(shot16.m))
    with pytest.raises(awe.AweError):                 # order 16: not built
        plan.step2_blocked(1)
    plan.close()
    plan = gpu_plan(shot, dt, src=np.zeros((0, 3)))
    with pytest.raises(awe.AweError):                 # no model yet
        plan.step2_blocked(1)
    plan.close()
