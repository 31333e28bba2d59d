"""GPU adjoint, dot-product test, gradient parity and checkpointing."""
import numpy as np
import pytest

import oracle
import synth
from helpers import dev, gpu_plan, host, log, oracle_problem, rel_l2, shot_dt, small_2d_shot, small_3d_shot

pytestmark = pytest.mark.gpu


def _dot_gpu(shot, seed):
    dt = shot_dt(shot)
    rng = np.random.default_rng(seed)
    nsrc, nrec = len(shot.src_coords), len(shot.rec_coords)
    x = synth.random_traces(rng, shot.nt, nsrc, shot.f0, dt)
    y = synth.random_traces(rng, shot.nt, nrec, shot.f0, dt)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    fx = host(plan.forward(dev(x)))
    fty, _ = plan.adjoint(dev(y))
    fty = host(fty)
    plan.close()
    xf, yf = x.astype(np.float32).astype(np.float64), y.astype(np.float32).astype(np.float64)
    lhs, rhs = float(np.sum(fx * yf)), float(np.sum(xf * fty))
    return abs(lhs - rhs) / max(abs(lhs), abs(rhs)), fty, (x, y, dt)


@pytest.mark.parametrize("kind,order", [("2d", 4), ("2d", 16), ("3d", 8), ("3d", 16)])
def test_dot_product(kind, order):
    shot = small_2d_shot(400 + order, order) if kind == "2d" else small_3d_shot(400 + order, order, nt=100)
    rel, fty, (x, y, dt) = _dot_gpu(shot, 5)
    log(f"case {shot.name}: dot-test rel {rel:.2e}")
    assert rel <= 1e-5
    # F^T y itself against the oracle
    ref = oracle.Operator(oracle_problem(shot, dt), shot.m).adjoint(y.astype(np.float32))["src_adj"]
    assert rel_l2(fty, ref) <= 1e-4
    assert np.all(fty[-1] == 0.0)


def _gradient_case(shot, K, seed=0):
    dt = shot_dt(shot)
    rng = np.random.default_rng(seed)
    w = shot.wavelet(dt)
    m_true = shot.m * (1.0 + 0.05 * synth.random_state(rng, shot.shape, 2.0))
    op_true = oracle.Operator(oracle_problem(shot, dt), m_true)
    d_obs = op_true.forward(w)["traces"].astype(np.float32)
    return dt, w, d_obs


@pytest.mark.parametrize("kind,order,K", [("2d", 4, 25), ("2d", 16, 7), ("3d", 8, 10), ("3d", 4, 33)])
def test_gradient_matches_oracle(kind, order, K):
    shot = small_2d_shot(500 + order, order, nt=200) if kind == "2d" else small_3d_shot(500 + order, order, nt=90)
    dt, w, d_obs = _gradient_case(shot, K)
    log(f"case {shot.name} K={K}")
    ref = oracle.Operator(oracle_problem(shot, dt), shot.m).gradient(w.astype(np.float32), d_obs)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    import paper_1608_08658_amd as awe
    tr = plan.forward(dev(w), ckpt_every=K)
    phi, resid = awe.misfit(tr, dev(d_obs))
    _, g = plan.adjoint(resid, want_src_adj=False, want_grad=True)
    g = host(g)
    gp = host(plan.gradient_padded())
    plan.close()
    e_g, e_gp = rel_l2(g, ref["grad"]), rel_l2(gp, ref["grad_pad"])
    log(f"  phi gpu {phi:.6e} oracle {ref['phi']:.6e}; grad rel {e_g:.2e} padded {e_gp:.2e}")
    assert phi == pytest.approx(ref["phi"], rel=1e-4)
    assert e_g <= 1e-4 and e_gp <= 1e-4


def test_gradient_is_independent_of_checkpoint_interval():
    # Recomputed segments repeat the forward's exact arithmetic, so every K
    # gives the same gradient bit for bit.
    shot = small_3d_shot(600, 8, nt=70)
    dt, w, d_obs = _gradient_case(shot, 1)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    import paper_1608_08658_amd as awe
    outs = []
    for K in (1, 2, 9, 69, 70, 200):
        tr = plan.forward(dev(w), ckpt_every=K)
        _, resid = awe.misfit(tr, dev(d_obs))
        _, g = plan.adjoint(resid, want_src_adj=False, want_grad=True)
        outs.append(host(g))
    plan.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_gradient_matches_oracle_finite_differences():
    # <g, dm> against a central difference of the FP64 oracle misfit.
    shot = small_2d_shot(700, 8, nt=200)
    dt, w, d_obs = _gradient_case(shot, 1, seed=3)
    rng = np.random.default_rng(11)
    dm = synth.random_state(rng, shot.shape, 3.0) * 0.01 * shot.m.mean()
    eps = 1e-2
    w32 = w.astype(np.float32)
    def phi(m):
        return oracle.misfit(oracle.Operator(oracle_problem(shot, dt), m).forward(w32)["traces"], d_obs)
    fd = (phi(shot.m + eps * dm) - phi(shot.m - eps * dm)) / (2 * eps)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    import paper_1608_08658_amd as awe
    tr = plan.forward(dev(w32), ckpt_every=20)
    _, resid = awe.misfit(tr, dev(d_obs))
    _, g = plan.adjoint(resid, want_src_adj=False, want_grad=True)
    gdm = float(np.sum(host(g) * dm))
    plan.close()
    log(f"  <g,dm> gpu {gdm:.6e}  oracle FD {fd:.6e}")
    assert gdm == pytest.approx(fd, rel=1e-3)


def test_gradient_without_checkpoints_is_a_state_error():
    shot = small_2d_shot(800, 4, nt=40)
    dt = shot_dt(shot)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    plan.forward(dev(shot.wavelet(dt)), ckpt_every=0)
    import torch
    import paper_1608_08658_amd as awe
    with pytest.raises(awe.AweError) as e:
        plan.adjoint(torch.zeros((shot.nt, len(shot.rec_coords)), device="cuda"), want_grad=True)
    assert e.value.status == -4


def test_reciprocity():
    shot = small_3d_shot(900, 8, nt=90)
    dt = shot_dt(shot)
    a = shot.src_coords[0]
    b = shot.rec_coords[3]
    w = shot.wavelet(dt)[:, :1]
    def trace(s, r):
        plan = gpu_plan(shot, dt, src=[s], rec=[r])
        plan.set_model(dev(shot.m))
        out = host(plan.forward(dev(w)))[:, 0]
        plan.close()
        return out
    ab, ba = trace(a, b), trace(b, a)
    e = rel_l2(ab, ba)
    log(f"  reciprocity rel {e:.2e}")
    assert e <= 1e-4


def test_misfit_matches_numpy():
    import paper_1608_08658_amd as awe
    rng = np.random.default_rng(1)
    a = rng.standard_normal((777, 33)).astype(np.float32)
    b = rng.standard_normal((777, 33)).astype(np.float32)
    phi, r = awe.misfit(dev(a), dev(b))
    ref = 0.5 * np.sum((a.astype(np.float64) - b) ** 2)
    assert phi == pytest.approx(ref, rel=1e-12)
    assert np.array_equal(host(r), (a - b).astype(np.float64))
