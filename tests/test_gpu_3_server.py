"""The continuous-batching shot server: results in the mix equal results alone,
admission respects the memory budget, a bad request fails alone, and
degenerate requests (one sample, no sources, no receivers) complete."""
import numpy as np
import pytest

import synth
from helpers import dev, gpu_plan, host, log, shot_dt

pytestmark = pytest.mark.gpu


def _requests(seed, count, scale):
    shots = synth.serving_requests(seed, count, scale=scale)
    out = []
    for s in shots:
        dt = float(shot_dt(s))
        out.append((s, dt, s.wavelet(dt).astype(np.float32)))
    return out


def _geom(shot, dt):
    import paper_1608_08658_amd as awe
    return awe.make_geometry(shape=shot.shape, spacing=shot.spacing, space_order=shot.order, nbl=shot.nbl, dt=dt,
                             nt=shot.nt, src_coords=shot.src_coords, rec_coords=shot.rec_coords,
                             damp_power=shot.damp_power, damp_R=shot.damp_R, damp_vref=shot.damp_vref)


def _alone(shot, dt, w):
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    tr = host(plan.forward(dev(w)))
    plan.close()
    return tr


def test_results_in_the_mix_equal_results_alone():
    import paper_1608_08658_amd as awe
    reqs = _requests(41, 8, scale=0.12)
    srv = awe.Server(hbm_fraction=0.5, chunk_steps=16, max_active=4)
    tickets = []
    for shot, dt, w in reqs:
        t, tr = srv.submit(_geom(shot, dt), shot.m, w)
        tickets.append((t, tr))
    for t, _ in tickets:
        srv.wait(t, timeout=300)
    stats = srv.stats()
    log(f"server stats {stats}")
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    for (shot, dt, w), (t, tr) in zip(reqs, tickets):
        st, times = srv.poll(t)
        assert st == 2
        assert times[0] <= times[1] <= times[2] <= times[3]
        alone = _alone(shot, dt, w)
        log(f"  {shot.name}: bitwise equal {np.array_equal(tr.astype(np.float64), alone)}")
        assert np.array_equal(tr.astype(np.float64), alone), shot.name
    # with nothing running, the retired requests' memory is freed
    import time
    t0 = time.time()
    while srv.stats()["bytes_reserved"] and time.time() - t0 < 30:
        time.sleep(0.01)
    assert srv.stats()["bytes_reserved"] == 0
    srv.close()


def test_admission_respects_budget(monkeypatch):
    import paper_1608_08658_amd as awe
    reqs = _requests(43, 6, scale=0.1)
    sizes = [awe.footprint(_geom(s, dt)) for s, dt, _ in reqs]
    budget = int(2.2 * max(sizes))
    monkeypatch.setenv("AWE_SERVER_BUDGET_BYTES", str(budget))
    srv = awe.Server(hbm_fraction=1.0, chunk_steps=8, max_active=16)
    tickets = [srv.submit(_geom(s, dt), s.m, w)[0] for s, dt, w in reqs]
    peak = 0
    import time
    t0 = time.time()
    while time.time() - t0 < 300:
        st = srv.stats()
        peak = max(peak, st["bytes_reserved"])
        if st["completed"] + st["failed"] == len(reqs):
            break
        time.sleep(0.002)
    st = srv.stats()
    log(f"budget {budget}, peak reserved {peak}, stats {st}")
    assert st["completed"] == len(reqs)
    assert peak <= budget
    srv.close()


def test_bad_request_fails_alone():
    import paper_1608_08658_amd as awe
    reqs = _requests(47, 3, scale=0.1)
    srv = awe.Server(hbm_fraction=0.5, chunk_steps=8, max_active=4)
    good = [srv.submit(_geom(s, dt), s.m, w)[0] for s, dt, w in reqs]
    s, dt, w = reqs[0]
    bad = srv.submit(_geom(s, 1.5 * dt / s.dt_factor), s.m, w)[0]      # above the stability limit
    for t in good:
        srv.wait(t, timeout=300)
    with pytest.raises(awe.AweError):
        srv.wait(bad, timeout=300)
    state, _ = srv.poll(bad)
    assert state == 3
    assert srv.stats()["completed"] == len(good)
    srv.close()


def test_oversized_request_is_rejected_at_submit(monkeypatch):
    import paper_1608_08658_amd as awe
    monkeypatch.setenv("AWE_SERVER_BUDGET_BYTES", "4096")
    srv = awe.Server(hbm_fraction=1.0, chunk_steps=8, max_active=2)
    s, dt, w = _requests(49, 1, scale=0.1)[0]
    with pytest.raises(awe.AweError) as e:
        srv.submit(_geom(s, dt), s.m, w)
    assert e.value.status == -2
    srv.close()


def test_degenerate_requests_complete():
    # one sample (no step), no sources, no receivers, from a 2-D and a 3-D
    # request, all in one server: each completes, with traces of its shape,
    # zero where no step is taken or nothing is injected
    import paper_1608_08658_amd as awe
    base = _requests(51, 2, scale=0.1)
    srv = awe.Server(hbm_fraction=0.5, chunk_steps=4, max_active=4)
    cases = []
    for shot, dt, w in base:
        one_shot = synth.Shot(shot.name + "-nt1", shot.shape, shot.spacing, shot.order, shot.nbl, 1, shot.m,
                              shot.src_coords, shot.rec_coords, shot.f0, damp_vref=shot.damp_vref)
        cases.append((one_shot, dt, w[:1]))
        nosrc = synth.Shot(shot.name + "-nosrc", shot.shape, shot.spacing, shot.order, shot.nbl, 9, shot.m,
                           np.zeros((0, len(shot.shape))), shot.rec_coords, shot.f0, damp_vref=shot.damp_vref)
        cases.append((nosrc, dt, np.zeros((9, 0), np.float32)))
        norec = synth.Shot(shot.name + "-norec", shot.shape, shot.spacing, shot.order, shot.nbl, 9, shot.m,
                           shot.src_coords, np.zeros((0, len(shot.shape))), shot.f0, damp_vref=shot.damp_vref)
        cases.append((norec, dt, w[:9]))
    tickets = []
    for shot, dt, w in cases:
        tickets.append(srv.submit(_geom(shot, dt), shot.m, w))
    for (t, _), (shot, _, _) in zip(tickets, cases):
        srv.wait(t, timeout=120)
        assert srv.poll(t)[0] == 2, shot.name
    for (t, tr), (shot, dt, w) in zip(tickets, cases):
        assert tr.shape == (shot.nt, len(shot.rec_coords)), shot.name
        if shot.nt == 1 or len(shot.src_coords) == 0:
            assert np.all(tr == 0.0), shot.name
    srv.close()


def _gradient_shot(seed, kind, order, nt):
    """A small shot, its true model (5% smooth perturbation) and d_obs from the
    oracle on the true model."""
    import oracle
    from helpers import oracle_problem, small_2d_shot, small_3d_shot
    shot = small_2d_shot(seed, order, nt=nt) if kind == "2d" else small_3d_shot(seed, order, nt=nt)
    dt = float(shot_dt(shot))
    rng = np.random.default_rng(seed)
    m_true = shot.m * (1.0 + 0.05 * synth.random_state(rng, shot.shape, 2.0))
    w = shot.wavelet(dt).astype(np.float32)
    d_obs = oracle.Operator(oracle_problem(shot, dt), m_true).forward(w)["traces"].astype(np.float32)
    return shot, dt, w, d_obs


def _gradient_alone(shot, dt, w, d_obs, K):
    """The same gradient through direct plan calls (forward, misfit, adjoint)."""
    import paper_1608_08658_amd as awe
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    tr = plan.forward(dev(w), ckpt_every=K)
    phi, resid = awe.misfit(tr, dev(d_obs))
    _, g = plan.adjoint(resid, want_src_adj=False, want_grad=True)
    out = host(g), host(tr), phi
    plan.close()
    return out


def test_gradient_requests_alone_in_the_mix_and_against_the_oracle():
    # Gradient requests among forward requests: each gradient, its traces and
    # misfit equal direct plan calls bit for bit (the server cuts the same
    # sweeps into chunks), every forward equals its shot alone, and the
    # gradient matches the oracle's.
    import torch
    import oracle
    import paper_1608_08658_amd as awe
    from helpers import oracle_problem, rel_l2
    K = 7
    # long enough that the direct wave reaches the receivers (a misfit of
    # numerical precursors alone would make the comparison meaningless)
    grads = [_gradient_shot(1301, "3d", 8, 60), _gradient_shot(1302, "2d", 4, 450), _gradient_shot(1303, "3d", 16, 60)]
    fwds = _requests(45, 5, scale=0.1)
    srv = awe.Server(hbm_fraction=0.5, chunk_steps=16, max_active=4)
    sub = []
    for i in range(max(len(grads), len(fwds))):
        if i < len(grads):
            shot, dt, w, d_obs = grads[i]
            g = torch.full(shot.shape, float("nan"), dtype=torch.float32, device="cuda")
            t, tr, phi = srv.submit_gradient(_geom(shot, dt), shot.m, w, d_obs, K, g)
            sub.append(("grad", i, t, tr, phi, g))
        if i < len(fwds):
            shot, dt, w = fwds[i]
            t, tr = srv.submit(_geom(shot, dt), shot.m, w)
            sub.append(("fwd", i, t, tr, None, None))
    for entry in sub:
        srv.wait(entry[2], timeout=300)
    stats = srv.stats()
    log(f"server stats {stats}")
    assert stats["completed"] == len(sub) and stats["failed"] == 0
    for kind, i, t, tr, phi, g in sub:
        if kind == "fwd":
            shot, dt, w = fwds[i]
            assert np.array_equal(tr.astype(np.float64), _alone(shot, dt, w)), shot.name
            continue
        shot, dt, w, d_obs = grads[i]
        g_alone, tr_alone, phi_alone = _gradient_alone(shot, dt, w, d_obs, K)
        g_srv = host(g)
        ref = oracle.Operator(oracle_problem(shot, dt), shot.m).gradient(w, d_obs)
        e = rel_l2(g_srv, ref["grad"])
        log(f"  gradient request {shot.name}: bitwise {np.array_equal(g_srv, g_alone)}, phi {phi[0]!r} vs "
            f"{phi_alone!r} (oracle {ref['phi']:.6e}), oracle gradient rel {e:.2e}")
        assert np.array_equal(g_srv, g_alone), shot.name
        assert np.array_equal(tr.astype(np.float64), tr_alone), shot.name
        assert phi[0] == phi_alone
        assert e <= 1e-4
    srv.close()


def test_served_gradients_summed_over_shots_against_the_oracle():
    # Three shots on one model (sources at different points): the server's
    # per-shot gradients summed in shot order on the device (FP64, one
    # rounding) equal that sum formed on the host, and the oracle's summed
    # gradient to 1e-4.
    import torch
    import oracle
    import paper_1608_08658_amd as awe
    from helpers import oracle_problem, rel_l2
    shot0, dt, w, _ = _gradient_shot(1401, "3d", 8, 60)
    rng = np.random.default_rng(1401)
    m_true = shot0.m * (1.0 + 0.05 * synth.random_state(rng, shot0.shape, 2.0))
    span = np.array([(n - 1) * h for n, h in zip(shot0.shape, shot0.spacing)])
    K = 9
    srv = awe.Server(hbm_fraction=0.5, chunk_steps=10, max_active=2)
    grads, tickets, ref_sum = [], [], None
    for k, frac in enumerate(([0.2, 0.3, 0.4], [0.25, 0.7, 0.6], [0.3, 0.5, 0.15])):
        import copy
        shot = copy.copy(shot0)
        shot.src_coords = np.array([np.array(frac) * span])
        op_true = oracle.Operator(oracle_problem(shot, dt), m_true)
        d_obs = op_true.forward(w)["traces"].astype(np.float32)
        ref = oracle.Operator(oracle_problem(shot, dt), shot.m).gradient(w, d_obs)["grad"]
        ref_sum = ref if ref_sum is None else ref_sum + ref
        g = torch.empty(shot.shape, dtype=torch.float32, device="cuda")
        tickets.append(srv.submit_gradient(_geom(shot, dt), shot.m, w, d_obs, K, g, want_traces=False)[0])
        grads.append(g)
    for t in tickets:
        srv.wait(t, timeout=300)
    srv.close()
    total = host(awe.sum_fields(grads))
    on_host = sum(host(g) for g in grads).astype(np.float32).astype(np.float64)
    e = rel_l2(total, ref_sum)
    log(f"  sum of 3 shots: oracle rel {e:.2e}, equal to the host FP64 sum {np.array_equal(total, on_host)}")
    assert np.array_equal(total, on_host)
    assert e <= 1e-4


def test_gradient_request_arguments_and_budget(monkeypatch):
    import torch
    import paper_1608_08658_amd as awe
    shot, dt, w, d_obs = _gradient_shot(1501, "3d", 8, 30)
    g = torch.empty(shot.shape, dtype=torch.float32, device="cuda")
    srv = awe.Server(hbm_fraction=0.5, chunk_steps=8, max_active=2)
    with pytest.raises(awe.AweError) as e:
        srv.submit_gradient(_geom(shot, dt), shot.m, w, d_obs, 0, g)
    assert e.value.status == -1
    srv.close()
    fp = awe.footprint(_geom(shot, dt), 5)
    monkeypatch.setenv("AWE_SERVER_BUDGET_BYTES", str(fp))     # below footprint + inputs
    srv = awe.Server(hbm_fraction=1.0, chunk_steps=8, max_active=2)
    with pytest.raises(awe.AweError) as e:
        srv.submit_gradient(_geom(shot, dt), shot.m, w, d_obs, 5, g)
    assert e.value.status == -2
    srv.close()


def test_repeated_gradient_requests_reuse_pooled_buffers_bit_for_bit():
    # One request at a time: every later request of the same grid takes the
    # earlier ones' retired buffers from the server's pool (its checkpoint
    # fields among them) and must give the same bits as the first and as
    # direct plan calls; with no work left the pool is freed.
    import torch
    import time
    import paper_1608_08658_amd as awe
    shot, dt, w, d_obs = _gradient_shot(1601, "3d", 8, 60)
    K = 6
    g_alone, tr_alone, phi_alone = _gradient_alone(shot, dt, w, d_obs, K)
    srv = awe.Server(hbm_fraction=0.5, chunk_steps=9, max_active=1)
    grads = [torch.full(shot.shape, float("nan"), dtype=torch.float32, device="cuda") for _ in range(3)]
    subs = [srv.submit_gradient(_geom(shot, dt), shot.m, w, d_obs, K, g) for g in grads]
    for t, _, _ in subs:
        srv.wait(t, timeout=300)
    for (t, tr, phi), g in zip(subs, grads):
        assert np.array_equal(host(g), g_alone)
        assert np.array_equal(tr.astype(np.float64), tr_alone)
        assert phi[0] == phi_alone
    t0 = time.time()
    while srv.stats()["bytes_reserved"] and time.time() - t0 < 30:
        time.sleep(0.01)
    assert srv.stats()["bytes_reserved"] == 0
    srv.close()


@pytest.mark.parametrize("max_active", [1, 2])
def test_requests_set_up_ahead_start_in_arrival_order(max_active):
    # with max_active requests running, the next one is set up ahead on a
    # host thread of its own; requests must still start in arrival order
    # (nothing is admitted past the one set up ahead) and give the bits they
    # give alone
    import paper_1608_08658_amd as awe
    reqs = _requests(47, 6, scale=0.1)
    srv = awe.Server(hbm_fraction=0.5, chunk_steps=8, max_active=max_active)
    subs = [srv.submit(_geom(shot, dt), shot.m, w) for shot, dt, w in reqs]
    for t, _ in subs:
        srv.wait(t, timeout=300)
    assert srv.stats()["completed"] == len(reqs) and srv.stats()["failed"] == 0
    times = [srv.poll(t)[1] for t, _ in subs]
    for i, tm in enumerate(times):
        log(f"  request {i}: admitted {tm[1]:.4f} started {tm[2]:.4f} done {tm[3]:.4f}")
        assert tm[0] <= tm[1] <= tm[2] <= tm[3]
    starts = [tm[2] for tm in times]
    assert starts == sorted(starts)
    # at most max_active + 1 requests are admitted and not done: request j is
    # admitted only after j - max_active of the earlier ones are done
    for j in range(max_active + 1, len(times)):
        done_before = sum(1 for k in range(j) if times[k][3] <= times[j][1])
        assert done_before >= j - max_active, (j, done_before)
    for (shot, dt, w), (t, tr) in zip(reqs, subs):
        assert np.array_equal(tr.astype(np.float64), _alone(shot, dt, w)), shot.name
    srv.close()
