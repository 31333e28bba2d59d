"""Binomial checkpointing on the GPU: the schedule only decides which
forward states are kept and which are recomputed, and a recomputed state
repeats the forward's exact arithmetic, so traces, F^T and the gradient must
equal those of periodic checkpointing bit for bit, for every number of
snapshots; the gradient is also checked against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from helpers import dev, gpu_plan, host, log, oracle_problem, rel_l2, shot_dt, small_2d_shot, small_3d_shot

pytestmark = pytest.mark.gpu


def _case(shot, seed=0, amp=0.05):
    dt = shot_dt(shot)
    rng = np.random.default_rng(seed)
    w = shot.wavelet(dt).astype(np.float32)
    m_true = shot.m * (1.0 + amp * synth.random_state(rng, shot.shape, 2.0))
    d_obs = oracle.Operator(oracle_problem(shot, dt), m_true).forward(w)["traces"].astype(np.float32)
    return dt, w, d_obs


def _run(plan, w, d_obs, K=None, snaps=None):
    import paper_1608_08658_amd as awe
    tr = plan.forward(dev(w), ckpt_every=K or 0, snapshots=snaps)
    _, resid = awe.misfit(tr, dev(d_obs))
    src_adj, g = plan.adjoint(resid, want_src_adj=True, want_grad=True)
    return host(tr), host(src_adj), host(g), plan.info()["bytes"]


@pytest.mark.parametrize("kind,order", [("2d", 4), ("3d", 8), ("3d", 16)])
def test_binomial_equals_periodic_bitwise(kind, order):
    import paper_1608_08658_amd as awe
    shot = small_2d_shot(700 + order, order, nt=160) if kind == "2d" else small_3d_shot(700 + order, order, nt=75)
    dt, w, d_obs = _case(shot)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    tr0, sa0, g0, _ = _run(plan, w, d_obs, K=9)
    for s in (0, 1, 2, 5, 13, shot.nt):
        tr, sa, g, held = _run(plan, w, d_obs, snaps=s)
        steps, fields = awe.binomial_cost(shot.nt, s)
        log(f"case {shot.name} snapshots {s}: {steps} forward steps, {fields} fields, {held} bytes held")
        assert np.array_equal(tr, tr0)
        assert np.array_equal(sa, sa0)
        assert np.array_equal(g, g0), s
    plan.close()


def test_binomial_gradient_matches_oracle():
    shot = small_3d_shot(720, 8, nt=90)
    dt, w, d_obs = _case(shot)
    op = oracle.Operator(oracle_problem(shot, dt), shot.m)
    fwd = op.forward(w, keep=True)
    resid = (fwd["traces"] - d_obs).astype(np.float32)
    g_ref = oracle.fold_padding(op.adjoint(resid, history=fwd["history"])["grad_pad"], shot.nbl)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    plan.forward(dev(w), snapshots=4)
    _, g = plan.adjoint(dev(resid), want_src_adj=False, want_grad=True)
    e = rel_l2(host(g), g_ref)
    log(f"case {shot.name} snapshots 4: gradient rel {e:.2e}")
    assert e <= 1e-4
    plan.close()


def test_binomial_autograd_and_state_rules():
    import torch
    import paper_1608_08658_amd as awe
    shot = small_2d_shot(730, 8, nt=120)
    dt, w, d_obs = _case(shot)
    plan = gpu_plan(shot, dt)
    grads = []
    for snaps in (None, 6):
        m = torch.tensor(shot.m, dtype=torch.float32, device="cuda", requires_grad=True)
        wt = torch.tensor(w, device="cuda", requires_grad=True)
        tr = awe.Gradient.apply(m, wt, plan, 10, snaps)
        loss = 0.5 * ((tr - dev(d_obs)) ** 2).sum()
        loss.backward()
        grads.append((host(m.grad), host(wt.grad)))
    assert np.array_equal(grads[0][0], grads[1][0]) and np.array_equal(grads[0][1], grads[1][1])
    # the schedule is consumed by its gradient: a second one is a state error
    plan.set_model(dev(shot.m))
    tr = plan.forward(dev(w), snapshots=3)
    _, resid = awe.misfit(tr, dev(d_obs))
    _, g1 = plan.adjoint(resid, want_src_adj=False, want_grad=True)
    with pytest.raises(awe.AweError) as e:
        plan.adjoint(resid, want_src_adj=False, want_grad=True)
    assert e.value.status == -4
    # F^T alone needs no stored states and leaves them alone
    plan.forward(dev(w), snapshots=3)
    plan.adjoint(resid, want_src_adj=True, want_grad=False)
    _, g2 = plan.adjoint(resid, want_src_adj=False, want_grad=True)
    assert np.array_equal(host(g1), host(g2))
    # switching back to periodic checkpoints releases the pool and still agrees
    b_binom = plan.info()["bytes"]
    plan.forward(dev(w), ckpt_every=10)
    _, g3 = plan.adjoint(resid, want_src_adj=False, want_grad=True)
    assert np.array_equal(host(g1), host(g3))
    b10 = plan.info()["bytes"]
    plan.forward(dev(w), ckpt_every=25)                # other storage; the old fields are released
    plan.forward(dev(w), ckpt_every=10)
    assert plan.info()["bytes"] == b10
    plan.forward(dev(w), snapshots=3)
    assert plan.info()["bytes"] == b_binom
    plan.close()


def test_binomial_gradient_crop_order16_2000_steps():
    # the 64^3 crop of the order-16 gradient workload at its full 2000 steps:
    # 20 stored states against checkpoints every 50 steps, bit for bit
    import paper_1608_08658_amd as awe
    shot = synth.config_3d_gradient_crop()
    m_true = shot.extra["m_true"]
    vmax = float(np.sqrt(1.0 / min(shot.m.min(), m_true.min())))
    dt = 0.5 * oracle.dt_max(shot.order, shot.spacing, vmax)
    w = shot.wavelet(dt).astype(np.float32)
    log(f"case {shot.name}: nt {shot.nt}")
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(m_true))
    d_obs = plan.forward(dev(w)).clone()
    plan.set_model(dev(shot.m))
    tr0 = plan.forward(dev(w), ckpt_every=shot.extra["checkpoint_every"])
    _, resid = awe.misfit(tr0, d_obs)
    _, g0 = plan.adjoint(resid, want_src_adj=False, want_grad=True)
    b0 = plan.info()["bytes"]
    tr1 = plan.forward(dev(w), snapshots=20)
    _, g1 = plan.adjoint(resid, want_src_adj=False, want_grad=True)
    b1 = plan.info()["bytes"]
    log(f"  periodic {b0 / 2**20:.0f} MiB, binomial {b1 / 2**20:.0f} MiB, "
        f"forward steps {awe.binomial_cost(shot.nt, 20)[0]}")
    assert np.array_equal(host(tr0), host(tr1))
    assert np.array_equal(host(g0), host(g1))
    assert b1 < b0
    plan.close()


@pytest.mark.parametrize("nt", [1, 2, 3])
def test_binomial_tiny_step_counts(nt):
    # no step, one step, two steps: the schedule degenerates, the gradient
    # (zero for nt = 1) and F^T still equal the periodic ones bit for bit
    shot = small_3d_shot(750 + nt, 4, nt=nt)
    dt = shot_dt(shot)
    w = (shot.wavelet(dt) * 1e3).astype(np.float32)
    rng = np.random.default_rng(nt)
    y = rng.standard_normal((nt, len(shot.rec_coords))).astype(np.float32)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    tr0 = host(plan.forward(dev(w), ckpt_every=1))
    sa0, g0 = plan.adjoint(dev(y), want_src_adj=True, want_grad=True)
    sa0, g0 = host(sa0), host(g0)
    for s in (0, 1, 5):
        tr = host(plan.forward(dev(w), snapshots=s))
        sa, g = plan.adjoint(dev(y), want_src_adj=True, want_grad=True)
        assert np.array_equal(tr, tr0) and np.array_equal(host(sa), sa0) and np.array_equal(host(g), g0), s
    if nt == 1:
        assert np.all(g0 == 0.0)
    plan.close()
