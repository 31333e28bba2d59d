"""Pins of the oracle's forward, adjoint and gradient (Sec. V.A-V.B)."""
import math

import numpy as np
import pytest

import synth
import oracle
from oracle import Operator, Problem, dt_max, misfit, weights_f64
from oracle.analytic import greens_2d, greens_3d


def _hetero_problem(seed, shape=(22, 26), nt=120, order=4, nbl=4, nsrc=2, nrec=7, h=(10.0, 12.0)):
    """A small heterogeneous problem with damping on, off-grid sources and receivers."""
    rng = np.random.default_rng(seed)
    ndim = len(shape)
    v = 1500.0 + 1000.0 * rng.random(shape)
    m = 1.0 / v ** 2
    dt = 0.6 * dt_max(order, h, v.max())
    span = np.array([(n - 1) * hh for n, hh in zip(shape, h)])
    src = rng.random((nsrc, ndim)) * span
    rec = rng.random((nrec, ndim)) * span
    p = Problem(shape, h, order, nbl, dt, nt, src, rec, damp_power=2, damp_vref=1500.0)
    return p, m, rng


@pytest.mark.parametrize("order", [4, 8])
def test_dispersion_closed_form(order):
    # Periodic, homogeneous, undamped: a plane wave cos(k.x) evolves exactly as
    # cos(w_h t_n), with 2 (1 - cos(w_h dt)) = v^2 dt^2 sum_a h_a^-2 (-c_0 - 2 sum_k c_k cos(k xi_a)),
    # xi_a = k_a h_a.  Anisotropic spacing catches axis/spacing mix-ups.
    shape = (16, 18, 20)
    h = (9.0, 11.0, 7.0)
    v = 2100.0
    modes = (3, 2, 5)
    dt = 0.8 * dt_max(order, h, v)
    nt = 300
    c = weights_f64(order)
    xi = [2 * math.pi * modes[a] / shape[a] for a in range(3)]
    lam = sum((-c[0] - 2 * sum(c[k] * math.cos(k * xi[a]) for k in range(1, len(c)))) / h[a] ** 2
              for a in range(3))
    w = math.acos(1.0 - 0.5 * (v * dt) ** 2 * lam) / dt
    grids = np.meshgrid(*[np.arange(shape[a]) for a in range(3)], indexing="ij")
    phase = sum(xi[a] * grids[a] for a in range(3))
    u0 = np.cos(phase)
    um1 = np.cos(phase) * math.cos(w * dt)
    p = Problem(shape, h, order, 0, dt, nt, np.zeros((0, 3)), np.zeros((0, 3)), periodic=True)
    out = Operator(p, np.full(shape, 1.0 / v ** 2)).forward(np.zeros((nt, 0)), state=(u0, um1))
    expect = np.cos(phase) * math.cos(w * (nt - 1) * dt)
    assert np.max(np.abs(out["u"] - expect)) < 1e-10


def _green_run_2d(h, dt, order=4, v=1500.0, f0=10.0, t_end=0.42, r=300.0):
    n = int(round(900.0 / h)) + 1
    shape = (n, n)
    c = (n - 1) * h / 2
    src = [[c, c]]
    rec = [[c, c + r]]
    nt = int(round(t_end / dt)) + 1
    dt = t_end / (nt - 1)
    s = synth.ricker_fn(f0, 1.5 / f0)
    p = Problem(shape, (h, h), order, 0, dt, nt, src, rec)
    tr = Operator(p, np.full(shape, 1.0 / v ** 2)).forward(s(np.arange(nt) * dt))["traces"][:, 0]
    t = np.arange(nt) * dt
    ref = greens_2d(r, t, v, s)
    return np.linalg.norm(tr - ref) / np.linalg.norm(ref)


@pytest.mark.slow
def test_convergence_to_analytic_2d_green():
    # Fixed Courant number: error dominated by O(dt^2) -> order -> 2.
    # dt ~ h^2: the O(h^4) spatial error shows -> order well above 2.
    # Reflections from the zero boundary (450 m away) arrive after the window.
    v, order = 1500.0, 4
    hs = (10.0, 5.0, 2.5)
    e_fixed = [_green_run_2d(h, 0.4 * dt_max(order, (h, h), v)) for h in hs]
    dt10 = 0.4 * dt_max(order, (10.0, 10.0), v)
    e_sq = [_green_run_2d(h, dt10 * (h / 10.0) ** 2) for h in hs]
    rate_fixed = math.log2(e_fixed[1] / e_fixed[2])
    rate_sq = math.log2(e_sq[1] / e_sq[2])
    assert e_fixed[0] < 1e-2
    assert rate_fixed > 1.6, e_fixed
    assert rate_sq > 2.8, e_sq


def test_analytic_3d_green():
    # One coarse 3-D run against u = s(t - r/v) / (4 pi r), before reflections.
    v, order, h, f0 = 1500.0, 8, 10.0, 12.0
    n = 51
    shape = (n, n, n)
    c = (n - 1) * h / 2
    r = 120.0
    dt = 0.4 * dt_max(order, (h,) * 3, v)
    t_end = 0.25
    nt = int(round(t_end / dt)) + 1
    s = synth.ricker_fn(f0, 1.5 / f0)
    p = Problem(shape, (h,) * 3, order, 0, dt, nt, [[c, c, c]], [[c, c, c + r], [c + r, c, c]])
    tr = Operator(p, np.full(shape, 1.0 / v ** 2)).forward(s(np.arange(nt) * dt))["traces"]
    ref = greens_3d(r, np.arange(nt) * dt, v, s)
    for j in range(2):
        assert np.linalg.norm(tr[:, j] - ref) / np.linalg.norm(ref) < 0.02


@pytest.mark.parametrize("shape,h", [((22, 26), (10.0, 12.0)), ((10, 12, 11), (10.0, 9.0, 11.0))])
def test_source_receiver_reciprocity(shape, h):
    # Swapping one source and one receiver gives the same trace, exactly up to
    # rounding, with heterogeneous m and the damping layer on.
    p, m, rng = _hetero_problem(7, shape=shape, h=h, nsrc=1, nrec=1, nt=90)
    a, b = p.src_coords[0], p.rec_coords[0]
    w = synth.ricker(25.0, p.dt, p.nt)
    def trace(src, rec):
        q = Problem(p.shape, p.spacing, p.order, p.nbl, p.dt, p.nt, [src], [rec], damp_power=2, damp_vref=1500.0)
        return Operator(q, m).forward(w)["traces"][:, 0]
    ab, ba = trace(a, b), trace(b, a)
    assert np.max(np.abs(ab - ba)) <= 1e-12 * np.max(np.abs(ab))


@pytest.mark.parametrize("shape,h,order", [((22, 26), (10.0, 12.0), 4), ((12, 10, 11), (10.0, 9.0, 11.0), 8)])
def test_dot_product(shape, h, order):
    # Eqs. (5)-(6): <F x, y> = <x, F^T y> for random band-limited x, y.
    p, m, rng = _hetero_problem(9, shape=shape, h=h, order=order)
    op = Operator(p, m)
    x = synth.random_traces(rng, p.nt, len(p.src_coords), 25.0, p.dt)
    y = synth.random_traces(rng, p.nt, len(p.rec_coords), 25.0, p.dt)
    fx = op.forward(x)["traces"]
    fty = op.adjoint(y)["src_adj"]
    lhs, rhs = np.sum(fx * y), np.sum(x * fty)
    assert abs(lhs - rhs) / max(abs(lhs), abs(rhs)) < 1e-13


def _grad_setup(seed=21):
    p, m, rng = _hetero_problem(seed, nrec=9, nt=110)
    m_true = m * (1.0 + 0.05 * synth.random_state(rng, p.shape, 2.0))
    w = synth.ricker(25.0, p.dt, p.nt)
    d_obs = Operator(p, m_true).forward(w)["traces"]
    dm = synth.random_state(rng, p.shape, 1.5) * (0.02 * m.mean())
    return p, m, w, d_obs, dm


def test_gradient_matches_central_differences():
    p, m, w, d_obs, dm = _grad_setup()
    g = Operator(p, m).gradient(w, d_obs)["grad"]
    eps = 1e-3
    fp = misfit(Operator(p, m + eps * dm).forward(w)["traces"], d_obs)
    fm = misfit(Operator(p, m - eps * dm).forward(w)["traces"], d_obs)
    fd = (fp - fm) / (2 * eps)
    assert abs(fd - np.sum(g * dm)) <= 1e-7 * abs(fd)


def test_gradient_taylor_orders():
    # Eqs. (7)-(8): the zeroth-order error falls like h, the first-order one like h^2.
    p, m, w, d_obs, dm = _grad_setup(23)
    op = Operator(p, m)
    res = op.gradient(w, d_obs)
    phi0, gdm = res["phi"], np.sum(res["grad"] * dm)
    hs = np.logspace(-6, 0, 13)
    e1, e2 = [], []
    for hh in hs:
        phi = misfit(Operator(p, m + hh * dm).forward(w)["traces"], d_obs)
        e1.append(abs(phi - phi0))
        e2.append(abs(phi - phi0 - hh * gdm))
    e1, e2 = np.array(e1), np.array(e2)
    # slopes over the part of the range where rounding does not dominate
    sel = (hs >= 1e-4) & (hs <= 1e-1)
    s1 = np.polyfit(np.log10(hs[sel]), np.log10(e1[sel]), 1)[0]
    s2 = np.polyfit(np.log10(hs[sel]), np.log10(e2[sel]), 1)[0]
    assert 0.9 < s1 < 1.1, s1
    assert 1.9 < s2 < 2.1, s2


@pytest.mark.parametrize("K", [1, 7, 25, 109, 110, 150])
def test_checkpointed_gradient_equals_full_storage(K):
    p, m, w, d_obs, _ = _grad_setup(29)
    op = Operator(p, m)
    full = op.gradient(w, d_obs)
    ck = op.gradient(w, d_obs, checkpoint_every=K)
    assert np.array_equal(full["grad_pad"], ck["grad_pad"])
    assert full["phi"] == ck["phi"]


def test_gradient_cancellation_free_form():
    # mu[n] - 2 mu[n+1] + mu[n+2] = C (L mu[n+1] + R^T y[n]) + (eta dt / D+) (mu[n+2] - mu[n+1])
    # (the form the GPU kernel accumulates); checked on the oracle's own arrays.
    p, m, w, d_obs, _ = _grad_setup(31)
    op = Operator(p, m)
    y = op.forward(w)["traces"] - d_obs
    rng = np.random.default_rng(0)
    mu1 = rng.standard_normal(p.padded_shape)
    mu2 = rng.standard_normal(p.padded_shape)
    mu = op.adjoint_step(mu1, mu2, y[40])
    from oracle.fd import laplacian
    from oracle.sparse import spread
    a = op.eta * p.dt / (op.m_pad + op.eta * p.dt / 2)
    rhs = op.C * (laplacian(mu1, p.spacing, p.order) + spread(p.padded_shape, *op.rec, y[40])) + a * (mu2 - mu1)
    assert np.max(np.abs((mu - 2 * mu1 + mu2) - rhs)) < 1e-12 * np.max(np.abs(mu))


def test_zero_wavelet_gives_zero_traces_and_first_sample_is_zero():
    p, m, rng = _hetero_problem(3)
    op = Operator(p, m)
    assert np.all(op.forward(np.zeros((p.nt, 2)))["traces"] == 0.0)
    tr = op.forward(synth.ricker(25.0, p.dt, p.nt)[:, None].repeat(2, 1))["traces"]
    assert np.all(tr[0] == 0.0) and np.any(tr[5] != 0.0)


def test_born_is_the_derivative_of_the_forward():
    # J dm against a central difference of the forward map (FP64).
    p, m, w, d_obs, dm = _grad_setup(41)
    op = Operator(p, m)
    jdm = op.born(w, dm)
    eps = 1e-4
    fp = Operator(p, m + eps * dm).forward(w)["traces"]
    fm = Operator(p, m - eps * dm).forward(w)["traces"]
    fd = (fp - fm) / (2 * eps)
    assert np.linalg.norm(jdm - fd) <= 1e-7 * np.linalg.norm(fd)


def test_born_dot_product_with_the_gradient():
    # <J dm, y> = <dm, J^T y>, J^T y being the adjoint-state gradient driven by y.
    p, m, w, d_obs, dm = _grad_setup(43)
    op = Operator(p, m)
    rng = np.random.default_rng(2)
    y = synth.random_traces(rng, p.nt, len(p.rec_coords), 25.0, p.dt)
    fwd = op.forward(w, keep=True)
    jty = oracle.fold_padding(op.adjoint(y, history=fwd["history"])["grad_pad"], p.nbl)
    lhs = np.sum(op.born(w, dm) * y)
    rhs = np.sum(dm * jty)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))
