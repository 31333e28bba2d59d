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


def _gradient_case(shot, K, seed=0, amp=0.05):
    dt = shot_dt(shot)
    rng = np.random.default_rng(seed)
    w = shot.wavelet(dt).astype(np.float32)
    m_true = shot.m * (1.0 + amp * synth.random_state(rng, shot.shape, 2.0))
    op_true = oracle.Operator(oracle_problem(shot, dt), m_true)
    d_obs = op_true.forward(w)["traces"].astype(np.float32)
    return dt, w, d_obs


def _gpu_gradient(shot, dt, w, K, resid=None, d_obs=None):
    """GPU forward with checkpoints, then the adjoint-state gradient driven by
    `resid` (given) or by traces - d_obs (computed on the device)."""
    import paper_1608_08658_amd as awe
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    tr = plan.forward(dev(w), ckpt_every=K)
    phi = None
    if resid is None:
        phi, r = awe.misfit(tr, dev(d_obs))
    else:
        r = dev(resid)
    _, g = plan.adjoint(r, want_src_adj=False, want_grad=True)
    out = host(g), host(plan.gradient_padded()), phi, host(tr)
    plan.close()
    return out


@pytest.mark.parametrize("kind,order,K", [("2d", 4, 25), ("2d", 16, 7), ("3d", 8, 10), ("3d", 4, 33),
                                          ("3d", 16, 1)])
def test_gradient_operator_matches_oracle(kind, order, K):
    # J^T applied to one and the same residual on both sides (the residual is
    # the oracle's, rounded to FP32): the adjoint-state gradient of Eq. (3).
    shot = small_2d_shot(500 + order, order, nt=200) if kind == "2d" else small_3d_shot(500 + order, order, nt=90)
    dt, w, d_obs = _gradient_case(shot, K)
    op = oracle.Operator(oracle_problem(shot, dt), shot.m)
    fwd = op.forward(w, keep=True)
    resid = (fwd["traces"] - d_obs).astype(np.float32)
    adj = op.adjoint(resid, history=fwd["history"])
    g_ref_pad = adj["grad_pad"]
    g_ref = oracle.fold_padding(g_ref_pad, shot.nbl)
    g, gp, _, _ = _gpu_gradient(shot, dt, w, K, resid=resid)
    e_g, e_gp = rel_l2(g, g_ref), rel_l2(gp, g_ref_pad)
    log(f"case {shot.name} K={K}: grad rel {e_g:.2e}, padded {e_gp:.2e}")
    assert e_g <= 1e-4 and e_gp <= 1e-4


@pytest.mark.parametrize("kind,order,amp", [("2d", 4, 0.05), ("3d", 8, 0.10)])
def test_gradient_end_to_end(kind, order, amp):
    # Inputs m, wavelet, d_obs -> misfit and gradient, the gradient to the
    # operator tolerance 1e-4.  The misfit is a sum of squared differences of
    # nearby traces, so an FP32 trace error eps is amplified by
    # kappa = |d| / |d - d_obs|: its bound is 2 eps kappa with eps = 1e-5 (the
    # forward's FP32 error level, a tenth of the trace tolerance).
    shot = small_2d_shot(510 + order, order, nt=200) if kind == "2d" else small_3d_shot(510 + order, order, nt=90)
    dt, w, d_obs = _gradient_case(shot, 10, amp=amp)
    ref = oracle.Operator(oracle_problem(shot, dt), shot.m).gradient(w, d_obs)
    kappa = np.linalg.norm(ref["traces"]) / np.linalg.norm(ref["traces"] - d_obs)
    g, gp, phi, tr = _gpu_gradient(shot, dt, w, 10, d_obs=d_obs)
    e_g = rel_l2(g, ref["grad"])
    e_phi = abs(phi - ref["phi"]) / ref["phi"]
    log(f"case {shot.name}: kappa {kappa:.1f}, traces {rel_l2(tr, ref['traces']):.2e}, "
        f"phi rel {e_phi:.2e}, grad rel {e_g:.2e}")
    assert rel_l2(tr, ref["traces"]) <= 1e-4
    assert e_phi <= 2e-5 * kappa
    assert e_g <= 1e-4


def test_autograd_matches_plan_calls():
    import torch
    import paper_1608_08658_amd as awe
    shot = small_2d_shot(520, 8, nt=150)
    dt, w, d_obs = _gradient_case(shot, 10)
    plan = gpu_plan(shot, dt)
    m = torch.tensor(shot.m, dtype=torch.float32, device="cuda", requires_grad=True)
    wt = torch.tensor(w, device="cuda", requires_grad=True)
    tr = awe.Gradient.apply(m, wt, plan, 15)
    loss = 0.5 * ((tr - dev(d_obs)) ** 2).sum()
    loss.backward()
    g_auto, gw_auto = host(m.grad), host(wt.grad)
    # the same through the plan
    plan.set_model(dev(shot.m))
    tr2 = plan.forward(dev(w), ckpt_every=15)
    resid = tr2 - dev(d_obs)
    src_adj, g = plan.adjoint(resid.contiguous(), want_src_adj=True, want_grad=True)
    assert np.array_equal(host(tr.detach()), host(tr2))
    assert np.array_equal(g_auto, host(g))
    assert np.array_equal(gw_auto, host(src_adj))
    plan.close()


def test_autograd_refuses_a_replaced_forward():
    # A plan holds one forward state.  Two graphs built on one plan: the
    # earlier one's backward must fail (AWE_ESTATE) rather than differentiate
    # the later forward; the later one's backward equals direct plan calls.
    import torch
    import paper_1608_08658_amd as awe
    shot = small_2d_shot(521, 8, nt=120)
    dt, w, d_obs = _gradient_case(shot, 10)
    plan = gpu_plan(shot, dt)
    m1 = torch.tensor(shot.m, dtype=torch.float32, device="cuda", requires_grad=True)
    m2 = torch.tensor(shot.m * 1.01, dtype=torch.float32, device="cuda", requires_grad=True)
    wt = torch.tensor(w, device="cuda", requires_grad=True)
    tr1 = awe.Gradient.apply(m1, wt, plan, 15)
    tr2 = awe.Gradient.apply(m2, wt, plan, 15)
    with pytest.raises(awe.AweError) as e:
        (0.5 * ((tr1 - dev(d_obs)) ** 2).sum()).backward()
    assert e.value.status == -4
    log(f"  stale backward refused: {e.value}")
    (0.5 * ((tr2 - dev(d_obs)) ** 2).sum()).backward()
    g_auto = host(m2.grad)
    plan.set_model(dev(shot.m * 1.01))
    tr = plan.forward(dev(w), ckpt_every=15)
    fid = plan.forward_id()
    _, g = plan.adjoint((tr - dev(d_obs)).contiguous(), want_src_adj=False, want_grad=True, forward_id=fid)
    assert np.array_equal(g_auto, host(g))
    # periodic checkpoints survive a gradient: the same id serves a second one
    _, g2 = plan.adjoint((tr - dev(d_obs)).contiguous(), want_src_adj=False, want_grad=True, forward_id=fid)
    assert np.array_equal(host(g2), host(g))
    plan.forward(dev(w), ckpt_every=0)
    with pytest.raises(awe.AweError) as e:
        plan.adjoint((tr - dev(d_obs)).contiguous(), want_src_adj=True, forward_id=fid)
    assert e.value.status == -4
    plan.close()


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
    # the residual is formed in FP32 (as stored), its square summed in FP64
    r32 = (a - b).astype(np.float64)
    ref = 0.5 * np.sum(r32 * r32)
    assert phi == pytest.approx(ref, rel=1e-12)
    assert np.array_equal(host(r), (a - b).astype(np.float64))


@pytest.mark.parametrize("order", [8, 16])
def test_gradient_across_launch_shapes(monkeypatch, order):
    # Every workgroup shape and z-chunk computes the same arithmetic per point,
    # so the gradient (forward in that shape, then the adjoint with imaging in
    # it) is the same bit for bit; each is also J^T of the oracle's residual to
    # the operator tolerance.  The grid is wider than two 128-point tiles (with
    # a ragged tail), so the two-wavefront tiles (4: 128 x 8, 5: 128 x 16) meet
    # x seams between their wavefronts and between tiles, and the chunks below
    # the z extent meet z seams.  Steps that load one plane ahead run whole
    # rounds of 2M+1 planes unguarded and the rest of a chunk guarded: chunks
    # of 9 (order 8) and 17 or 34 planes (the order-16 imaging step) are whole
    # rounds only, the others end in a partial round.
    shot = small_3d_shot(610 + order, order, shape=(40, 46, 150), nt=40)
    K = 8
    dt, w, d_obs = _gradient_case(shot, K)
    op = oracle.Operator(oracle_problem(shot, dt), shot.m)
    fwd = op.forward(w, keep=True)
    resid = (fwd["traces"] - d_obs).astype(np.float32)
    g_ref = oracle.fold_padding(op.adjoint(resid, history=fwd["history"])["grad_pad"], shot.nbl)
    outs = []
    for cfg in ("0,9", "1,31", "3,56", "4,13", "4,28", "5,21", "5,84", "2,17", "1,34"):
        monkeypatch.setenv("AWE_TILE", cfg)
        plan = gpu_plan(shot, dt)
        plan.set_model(dev(shot.m))
        plan.forward(dev(w), ckpt_every=K)
        _, g = plan.adjoint(dev(resid), want_src_adj=False, want_grad=True)
        info = plan.info()
        assert info["forward_shape"] == info["imaging_shape"] == tuple(int(v) for v in cfg.split(","))
        outs.append(host(g))
        plan.close()
        e = rel_l2(outs[-1], g_ref)
        log(f"case {shot.name} shape {cfg}: gradient rel {e:.2e}")
        assert e <= 1e-4
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
