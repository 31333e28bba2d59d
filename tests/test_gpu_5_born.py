"""Linearised (Born) modelling J dm on the GPU."""
import numpy as np
import pytest

import oracle
import synth
from helpers import dev, gpu_plan, host, log, oracle_problem, rel_l2, shot_dt, small_2d_shot, small_3d_shot

pytestmark = pytest.mark.gpu


def _case(kind, order, seed):
    shot = small_2d_shot(seed, order, nt=200) if kind == "2d" else small_3d_shot(seed, order, nt=90)
    dt = shot_dt(shot)
    rng = np.random.default_rng(seed)
    dm = (synth.random_state(rng, shot.shape, 2.0) * 0.05 * shot.m.mean()).astype(np.float32)
    return shot, dt, shot.wavelet(dt).astype(np.float32), dm


@pytest.mark.parametrize("kind,order", [("2d", 4), ("2d", 16), ("3d", 8), ("3d", 16)])
def test_born_matches_oracle(kind, order):
    shot, dt, w, dm = _case(kind, order, 800 + order)
    ref = oracle.Operator(oracle_problem(shot, dt), shot.m).born(w, dm)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    got = host(plan.born(dev(w), dev(dm)))
    plan.close()
    e = rel_l2(got, ref)
    log(f"case {shot.name}: Born rel {e:.2e}")
    assert np.all(got[0] == 0.0)
    assert e <= 1e-4


@pytest.mark.parametrize("kind,order", [("2d", 8), ("3d", 8)])
def test_born_dot_product_with_gradient(kind, order):
    # <J dm, y> = <dm, J^T y>: the GPU's linearised modelling against its
    # adjoint-state gradient driven by y.
    shot, dt, w, dm = _case(kind, order, 820 + order)
    rng = np.random.default_rng(3)
    y = synth.random_traces(rng, shot.nt, len(shot.rec_coords), shot.f0, dt).astype(np.float32)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    jdm = host(plan.born(dev(w), dev(dm)))
    plan.forward(dev(w), ckpt_every=17)
    _, jty = plan.adjoint(dev(y), want_src_adj=False, want_grad=True)
    jty = host(jty)
    plan.close()
    lhs = float(np.sum(jdm * y.astype(np.float64)))
    rhs = float(np.sum(dm.astype(np.float64) * jty))
    rel = abs(lhs - rhs) / max(abs(lhs), abs(rhs))
    log(f"case {shot.name}: Born dot test {rel:.2e}")
    assert rel <= 1e-5


def test_born_is_linear():
    # Doubling dm doubles every value except where intermediate values are
    # subnormal (they round at reduced precision), so the bound is relative.
    shot, dt, w, dm = _case("3d", 4, 840)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    a = host(plan.born(dev(w), dev(dm)))
    b = host(plan.born(dev(w), dev(2.0 * dm)))
    z = host(plan.born(dev(w), dev(0.0 * dm)))
    plan.close()
    assert rel_l2(b, 2.0 * a) <= 1e-6
    assert np.all(z == 0.0)


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_born_fused_point_operators_bitwise(monkeypatch, kind):
    # The background step injecting (into u and t) and the scattered step
    # sampling inside their own launches give exactly the separate-launch
    # results; the source sits on tile and chunk seams.
    shot, dt, w, dm = _case(kind, 8, 860)
    h = shot.spacing
    if kind == "3d":
        shot.src_coords = np.array([[(6.5 - shot.nbl) * h[0], (15.5 - shot.nbl) * h[1], (63.5 - shot.nbl) * h[2]]])
    else:
        shot.src_coords = np.array([[(15.5 - shot.nbl) * h[0], (63.5 - shot.nbl) * h[1]]])
    outs = []
    for fuse in (None, "0"):
        if fuse is None:
            monkeypatch.delenv("AWE_FUSE", raising=False)
        else:
            monkeypatch.setenv("AWE_FUSE", fuse)
        plan = gpu_plan(shot, dt)
        plan.set_model(dev(shot.m))
        outs.append(host(plan.born(dev(w), dev(dm))))
        plan.close()
    assert np.any(outs[0] != 0.0)
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("order", [2, 8, 16])
def test_born_one_sweep_bitwise_equal_to_two_launches(monkeypatch, order):
    # 3-D: the background and the scattered step in one sweep (t in a
    # register, the source injected into u and t inside the sweep) give the
    # bits of the save-t and born launches; the source cell straddles a tile
    # row seam (y 15/16) and a z-chunk seam, receivers sample du.
    shot, dt, w, dm = _case("3d", order, 870 + order)
    h = shot.spacing
    shot.src_coords = np.array([[(27.5 - shot.nbl) * h[0], (15.5 - shot.nbl) * h[1], (63.5 - shot.nbl) * h[2]]])
    monkeypatch.setenv("AWE_TILE", "1,28")
    outs = []
    for env in (None, "0"):
        if env is None:
            monkeypatch.delenv("AWE_BORN_FUSED", raising=False)
        else:
            monkeypatch.setenv("AWE_BORN_FUSED", env)
        plan = gpu_plan(shot, dt)
        plan.set_model(dev(shot.m))
        outs.append(host(plan.born(dev(w), dev(dm))))
        plan.close()
    log(f"order {order}: max |J dm| {np.abs(outs[0]).max():.3e}")
    assert np.any(outs[0] != 0.0)
    assert np.array_equal(outs[0], outs[1])
