"""GPU forward parity against the FP64 oracle (traces and wavefields, rel-L2 <= 1e-4)."""
import numpy as np
import pytest

import oracle
import synth
from helpers import dev, gpu_plan, host, log, oracle_problem, rel_l2, shot_dt, small_2d_shot, small_3d_shot

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _run_both(shot, dt=None):
    dt = dt or shot_dt(shot)
    w = shot.wavelet(dt)
    ref = oracle.Operator(oracle_problem(shot, dt), shot.m).forward(w)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    tr = plan.forward(dev(w))
    u, up = plan.get_state()
    out = host(tr), host(u), host(up)
    plan.close()
    return ref, out


def test_2d_101x101_order4_500_steps():
    shot = synth.config_2d_small()
    log(f"case {shot.name}")
    ref, (tr, u, up) = _run_both(shot)
    e_tr, e_u, e_up = rel_l2(tr, ref["traces"]), rel_l2(u, ref["u"]), rel_l2(up, ref["u_prev"])
    log(f"  traces {e_tr:.2e}  u[nt-1] {e_u:.2e}  u[nt-2] {e_up:.2e}")
    assert np.all(tr[0] == 0.0)
    assert e_tr <= TOL and e_u <= TOL and e_up <= TOL


@pytest.mark.parametrize("order", [2, 4, 8, 16])
def test_2d_orders(order):
    shot = small_2d_shot(100 + order, order)
    log(f"case {shot.name}")
    ref, (tr, u, _) = _run_both(shot)
    e_tr, e_u = rel_l2(tr, ref["traces"]), rel_l2(u, ref["u"])
    log(f"  traces {e_tr:.2e}  u {e_u:.2e}")
    assert e_tr <= TOL and e_u <= TOL


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12, 14, 16])
def test_3d_orders_multi_tile_ragged(order):
    shot = small_3d_shot(200 + order, order)
    log(f"case {shot.name} shape {shot.shape} nbl {shot.nbl}")
    ref, (tr, u, _) = _run_both(shot)
    e_tr, e_u = rel_l2(tr, ref["traces"]), rel_l2(u, ref["u"])
    log(f"  traces {e_tr:.2e}  u {e_u:.2e}")
    assert e_tr <= TOL and e_u <= TOL


@pytest.mark.parametrize("cfg", ["0,7", "1,16", "2,33", "3,100"])
def test_3d_every_launch_shape(cfg, monkeypatch):
    # Every workgroup shape and z-chunk length gives the same answer.
    monkeypatch.setenv("AWE_TILE", cfg)
    shot = small_3d_shot(300, 8, nt=60)
    log(f"case tile {cfg}")
    ref, (tr, u, _) = _run_both(shot)
    assert rel_l2(tr, ref["traces"]) <= TOL and rel_l2(u, ref["u"]) <= TOL


@pytest.mark.parametrize("cfg", ["0,5", "1,64"])
def test_2d_every_launch_shape(cfg, monkeypatch):
    monkeypatch.setenv("AWE_TILE", cfg)
    shot = small_2d_shot(301, 8, nt=120)
    ref, (tr, u, _) = _run_both(shot)
    assert rel_l2(tr, ref["traces"]) <= TOL and rel_l2(u, ref["u"]) <= TOL


def test_repeat_runs_are_bitwise_identical():
    shot = small_3d_shot(7, 8, nt=50)
    dt = shot_dt(shot)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    w = dev(shot.wavelet(dt))
    a = host(plan.forward(w))
    b = host(plan.forward(w))
    assert np.array_equal(a, b)


def test_forward_resumes_from_state_bitwise():
    # The state of the second-order recurrence is the pair (u[n], u[n-1]):
    # restarting from it reproduces an uninterrupted run exactly.
    shot = small_3d_shot(8, 4, nt=80)
    dt = shot_dt(shot)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    w = dev(shot.wavelet(dt))
    full = host(plan.forward(w))
    import torch
    tr = torch.zeros((shot.nt, len(shot.rec_coords)), dtype=torch.float32, device="cuda")
    z = torch.zeros(plan.padded, dtype=torch.float32, device="cuda")
    plan.set_state(z, z)
    plan.step(0, 30, w, tr)
    u, up = plan.get_state()
    plan.set_state(u, up)
    plan.step(30, shot.nt - 31, w, tr)
    assert np.array_equal(host(tr), full)


def _state_steps_sampled(shot, pts, seed=42, nsteps=3):
    """nsteps GPU steps from a seeded smooth random state, compared point by
    point with the oracle evaluated on small sub-blocks around the points."""
    dt = shot_dt(shot)
    rng = np.random.default_rng(seed)
    P = tuple(n + 2 * shot.nbl for n in shot.shape)
    u0 = synth.random_state(rng, P, 3.0).astype(np.float32)
    um = (u0 * 0.999).astype(np.float32)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    w = shot.wavelet(dt) * 1e3
    plan.set_state(dev(u0), dev(um))
    plan.step(0, nsteps, dev(w), None)
    u, _ = plan.get_state()
    u = host(u)
    log(f"  launch shape {plan.info()['forward_shape']}")
    plan.close()
    op = oracle.Operator(oracle_problem(shot, dt, nt=nsteps + 1), shot.m)
    r = nsteps * (shot.order // 2)
    from oracle.fd import laplacian
    from oracle.sparse import spread
    for p in pts:
        lo = [max(0, p[a] - r) for a in range(3)]
        hi = [min(P[a], p[a] + r + 1) for a in range(3)]
        sl = tuple(slice(lo[a], hi[a]) for a in range(3))
        cu, cp = u0[sl].astype(np.float64), um[sl].astype(np.float64)
        A, B, Cc = op.A[sl], op.B[sl], op.C[sl]
        # zero outside the true grid is exact; a cut inside the grid only
        # pollutes cells within r of the cut, which p never is.
        src_nodes, src_w = op.src
        for n in range(nsteps):
            q = spread(P, src_nodes, src_w, w[n]) / op.vol
            nxt = A * cu - B * cp + Cc * (laplacian(cu, shot.spacing, shot.order) + q[sl])
            cp, cu = cu, nxt
        want = cu[tuple(p[a] - lo[a] for a in range(3))]
        got = u[p]
        scale = max(abs(want), 1e-3 * np.max(np.abs(u0)))
        log(f"  point {p}: gpu {got:.7e} oracle {want:.7e}")
        assert abs(got - want) <= 1e-5 * scale, p


def _src_node(shot):
    return tuple(np.floor(shot.src_coords[0] / np.array(shot.spacing) + shot.nbl).astype(int))


def test_full_size_state_steps_sampled():
    # At the full 3-D forward size (256^3 + 40-point layer, order 8) and in the
    # launch shape the benchmark uses: three steps from a seeded smooth random
    # state, compared point by point with the oracle evaluated on small
    # sub-blocks around sampled points (corners, faces, the layer, tile seams,
    # the source).
    shot = synth.config_3d_forward(nt=4)
    P = tuple(n + 2 * shot.nbl for n in shot.shape)
    log(f"case full-size state steps {P}")
    pts = [(0, 0, 0), (P[0] - 1, P[1] - 1, P[2] - 1), (0, 170, 63), (335, 64, 128), (40, 40, 40),
           (167, 15, 16), (168, 16, 64), (200, 300, 335), (17, 200, 1), _src_node(shot), (100, 127, 191)]
    _state_steps_sampled(shot, pts)


@pytest.mark.parametrize("tile", [None, "3,30", "1,38"])
def test_full_size_paper_example_state_steps_sampled(tile, monkeypatch):
    # The paper's 3-D run (order 14, 150 x 281 x 281 computed: five 64-point x
    # tiles, the last holding 25 columns) in the autotuned shape and in the
    # shapes the tuner picks there: points at the corners, on z-chunk seams
    # (multiples of 30 and 38), on tile-row seams (multiples of 8 and 16), on
    # x-tile seams and in the ragged last x tile, in the layer, on the
    # receiver line and at the source.
    if tile is None:
        monkeypatch.delenv("AWE_TILE", raising=False)
    else:
        monkeypatch.setenv("AWE_TILE", tile)
    monkeypatch.delenv("AWE_AUTOTUNE", raising=False)
    shot = synth.config_paper_example()
    shot.nt = 4
    P = tuple(n + 2 * shot.nbl for n in shot.shape)
    log(f"case paper example state steps {P}, tile {tile}")
    pts = [(0, 0, 0), (P[0] - 1, P[1] - 1, P[2] - 1), (29, 15, 63), (30, 16, 64), (37, 8, 127), (38, 135, 128),
           (60, 128, 255), (75, 200, 256), (89, 271, 280), (90, 280, 270), (119, 47, 192), (120, 140, 191),
           (42, 140, 1), (42, 140, 279), (149, 0, 280), _src_node(shot)]
    _state_steps_sampled(shot, pts)


def _forward_with_env(monkeypatch, shot, dt, env):
    for k, v in env.items():
        if v is None:
            monkeypatch.delenv(k, raising=False)
        else:
            monkeypatch.setenv(k, v)
    plan = gpu_plan(shot, dt)
    plan.set_model(dev(shot.m))
    tr = host(plan.forward(dev(shot.wavelet(dt))))
    u, _ = plan.get_state()
    plan.close()
    return tr, host(u)


def test_every_launch_shape_is_bitwise_identical(monkeypatch):
    # Tiling changes where a neighbour value comes from (registers or LDS),
    # never the arithmetic of a point: all shapes agree bit for bit.
    shot = small_3d_shot(310, 8, nt=40)
    dt = shot_dt(shot)
    ref = None
    for cfg in ("0,7", "1,8", "1,16", "2,33", "3,100", "3,56", "4,9", "5,30"):
        out = _forward_with_env(monkeypatch, shot, dt, {"AWE_TILE": cfg})
        if ref is None:
            ref = out
        else:
            assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), cfg


def test_autotuned_plan_matches_forced_shape(monkeypatch):
    # 140^3 + 2 x 12 layer = 164^3 padded (> 4M points): the plan autotunes.
    rng = np.random.default_rng(5)
    shape = (140, 140, 140)
    v = synth.layered_velocity(shape, rng, nlayers=(3, 5))
    shot = synth.Shot("tune-140", shape, (10.0,) * 3, 8, 12, 30, 1.0 / v ** 2,
                      np.array([[300.0, 700.0, 700.0]]), np.array([[25.0, 100.0 + 7 * i, 900.0] for i in range(50)]),
                      20.0, damp_vref=float(v.min()))
    dt = shot_dt(shot)
    tuned = _forward_with_env(monkeypatch, shot, dt, {"AWE_TILE": None, "AWE_AUTOTUNE": None})
    forced = _forward_with_env(monkeypatch, shot, dt, {"AWE_TILE": "1,28"})
    assert np.array_equal(tuned[0], forced[0]) and np.array_equal(tuned[1], forced[1])


@pytest.mark.parametrize("order", [4, 16])
def test_autotuned_2d_plan_matches_forced_shape(monkeypatch, order):
    # 2-D grids from 64K points are tuned (zchunks down to 4 planes per wave)
    shot = small_2d_shot(320 + order, order, shape=(330, 290), nbl=12, nt=60)
    dt = shot_dt(shot)
    tuned = _forward_with_env(monkeypatch, shot, dt, {"AWE_TILE": None, "AWE_AUTOTUNE": None})
    for cfg in ("0,4", "1,8", "0,64"):
        forced = _forward_with_env(monkeypatch, shot, dt, {"AWE_TILE": cfg})
        assert np.array_equal(tuned[0], forced[0]) and np.array_equal(tuned[1], forced[1]), cfg


def test_nearby_3d_sizes_each_get_a_shape_with_the_same_results(monkeypatch):
    # plans made directly time their own size even next to a tuned nearby
    # size (the rule is checked on the CPU, tests/cpp/tune_policy_check.cpp);
    # whatever shape each takes, its traces equal a forced run of the
    # built-in shape bit for bit
    rng = np.random.default_rng(6)
    for n in (150, 156):
        shape = (n, n, n)
        v = synth.layered_velocity(shape, rng, nlayers=(3, 5))
        shot = synth.Shot(f"near-{n}", shape, (10.0,) * 3, 16, 12, 12, 1.0 / v ** 2,
                          np.array([[300.0, 700.0, 700.0]]), np.array([[25.0, 100.0, 900.0]]), 20.0,
                          damp_vref=float(v.min()))
        dt = shot_dt(shot)
        tuned = _forward_with_env(monkeypatch, shot, dt, {"AWE_TILE": None, "AWE_AUTOTUNE": None})
        forced = _forward_with_env(monkeypatch, shot, dt, {"AWE_TILE": None, "AWE_AUTOTUNE": "0"})
        log(f"n={n}: tuned and built-in shapes give equal traces")
        assert np.array_equal(tuned[0], forced[0]) and np.array_equal(tuned[1], forced[1])


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_fused_point_operators_bitwise(monkeypatch, kind):
    # A plain step with few source nodes injects and samples inside the
    # stencil launch; it must give exactly what the separate point-operator
    # launch gives.  The source sits on an x-tile seam, a y-tile seam (3-D)
    # and a z-chunk seam of the forced shapes, so its nodes belong to
    # different workgroups.
    if kind == "3d":
        shot = small_3d_shot(330, 8, nt=50)      # padded 52 x 58 x 102, nbl 6
        h = shot.spacing
        shot.src_coords = np.array([[(6.5 - 6) * h[0], (15.5 - 6) * h[1], (63.5 - 6) * h[2]]])
        cfgs = ("3,7", "0,7", "1,16", "4,7", "5,7")
    else:
        shot = small_2d_shot(331, 8, nt=80)      # padded 170 x 190, nbl 10
        h = shot.spacing
        shot.src_coords = np.array([[(15.5 - 10) * h[0], (63.5 - 10) * h[1]]])
        cfgs = ("0,4", "1,16")
    dt = shot_dt(shot)
    for cfg in cfgs:
        fused = _forward_with_env(monkeypatch, shot, dt, {"AWE_TILE": cfg, "AWE_FUSE": None})
        split = _forward_with_env(monkeypatch, shot, dt, {"AWE_TILE": cfg, "AWE_FUSE": "0"})
        assert np.any(fused[0] != 0.0)
        assert np.array_equal(fused[0], split[0]) and np.array_equal(fused[1], split[1]), cfg
