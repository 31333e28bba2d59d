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
