"""Order-16 FWI gradient on the 64^3 crop of the 400^3 problem (h = 12.5 m,
2000 time samples, checkpoints every 50 steps) against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import paper_1608_08658_amd as awe
import synth
from helpers import dev, gpu_plan, host, log, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu


def test_order16_gradient_crop_2000_steps():
    shot = synth.config_3d_gradient_crop()
    K = shot.extra["checkpoint_every"]
    m_true = shot.extra["m_true"]
    vmax = float(np.sqrt(1.0 / min(shot.m.min(), m_true.min())))
    dt = 0.5 * oracle.dt_max(shot.order, shot.spacing, vmax)
    w = shot.wavelet(dt).astype(np.float32)
    log(f"case {shot.name}: padded {[n + 2 * shot.nbl for n in shot.shape]}, nt {shot.nt}, K {K}, dt {dt:.3e}")
    prob = oracle_problem(shot, dt)
    d_obs = oracle.Operator(prob, m_true, backend="c").forward(w)["traces"].astype(np.float32)
    op = oracle.Operator(prob, shot.m, backend="c")
    ref = op.gradient(w, d_obs, checkpoint_every=K)
    log(f"  oracle phi {ref['phi']:.6e}")

    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    tr = plan.forward(dev(w), ckpt_every=K)
    phi, resid = awe.misfit(tr, dev(d_obs))
    _, g = plan.adjoint(resid, want_src_adj=False, want_grad=True)
    g = host(g)
    # the operator alone: J^T on the oracle's own residual
    resid_ref = (ref["traces"] - d_obs).astype(np.float32)
    plan.forward(dev(w), ckpt_every=K)
    _, g_op = plan.adjoint(dev(resid_ref), want_src_adj=False, want_grad=True)
    g_op = host(g_op)
    plan.close()

    kappa = np.linalg.norm(ref["traces"]) / np.linalg.norm(ref["traces"] - d_obs)
    e_tr = rel_l2(host(tr), ref["traces"])
    e_op = rel_l2(g_op, ref["grad"])
    e_g = rel_l2(g, ref["grad"])
    e_phi = abs(phi - ref["phi"]) / ref["phi"]
    log(f"  traces {e_tr:.2e}; J^T on the same residual {e_op:.2e}; kappa {kappa:.1f}; "
        f"phi {e_phi:.2e}; gradient {e_g:.2e}")
    assert e_tr <= 1e-4
    assert e_op <= 1e-4
    assert e_phi <= 2e-5 * kappa
    assert e_g <= 1e-4
