"""Planted mistakes in the oracle (on the CPU) must each break at least one pin.

Every case patches one plausible error into the oracle for the duration of
the test and checks that the corresponding pin fails; together they show the
pins are not blind to dropped terms, wrong signs, wrong indices or
transposed operands.
"""
import math

import numpy as np
import pytest

import oracle.fd
import oracle.medium
import oracle.sparse
import oracle.wave
import synth
from oracle import Operator, Problem, dt_max, misfit, weights_f64
from oracle.analytic import greens_2d


def _green_err_2d(h=10.0, v=1500.0, order=4, f0=10.0, t_end=0.42, r=300.0):
    n = int(round(900.0 / h)) + 1
    c = (n - 1) * h / 2
    dt = 0.4 * dt_max(order, (h, h), v)
    nt = int(round(t_end / dt)) + 1
    dt = t_end / (nt - 1)
    s = synth.ricker_fn(f0, 1.5 / f0)
    p = Problem((n, n), (h, h), order, 0, dt, nt, [[c, c]], [[c, c + r]])
    tr = Operator(p, np.full((n, n), 1.0 / v ** 2)).forward(s(np.arange(nt) * dt))["traces"][:, 0]
    ref = greens_2d(r, np.arange(nt) * dt, v, s)
    return np.linalg.norm(tr - ref) / np.linalg.norm(ref)


def _dot_rel(order=4):
    rng = np.random.default_rng(9)
    shape, h = (22, 26), (10.0, 12.0)
    v = 1500.0 + 1000.0 * rng.random(shape)
    dt = 0.6 * dt_max(order, h, v.max())
    span = np.array([(n - 1) * hh for n, hh in zip(shape, h)])
    p = Problem(shape, h, order, 4, dt, 100, rng.random((2, 2)) * span, rng.random((7, 2)) * span,
                damp_power=2, damp_vref=1500.0)
    op = Operator(p, 1.0 / v ** 2)
    x = synth.random_traces(rng, p.nt, 2, 25.0, dt)
    y = synth.random_traces(rng, p.nt, 7, 25.0, dt)
    lhs = np.sum(op.forward(x)["traces"] * y)
    rhs = np.sum(x * op.adjoint(y)["src_adj"])
    return abs(lhs - rhs) / max(abs(lhs), abs(rhs))


def _grad_rel():
    rng = np.random.default_rng(21)
    shape, h = (20, 24), (10.0, 12.0)
    v = 1500.0 + 1000.0 * rng.random(shape)
    m = 1.0 / v ** 2
    dt = 0.6 * dt_max(4, h, v.max())
    span = np.array([(n - 1) * hh for n, hh in zip(shape, h)])
    p = Problem(shape, h, 4, 4, dt, 100, rng.random((1, 2)) * span, rng.random((9, 2)) * span,
                damp_power=2, damp_vref=1500.0)
    w = synth.ricker(25.0, dt, p.nt)
    d_obs = Operator(p, m * (1 + 0.05 * synth.random_state(rng, shape))).forward(w)["traces"]
    dm = synth.random_state(rng, shape) * 0.02 * m.mean()
    g = Operator(p, m).gradient(w, d_obs)["grad"]
    eps = 1e-3
    fd = (misfit(Operator(p, m + eps * dm).forward(w)["traces"], d_obs)
          - misfit(Operator(p, m - eps * dm).forward(w)["traces"], d_obs)) / (2 * eps)
    return abs(fd - np.sum(g * dm)) / abs(fd)


def _absorb_err():
    h, v, order = 10.0, 1500.0, 4
    dt = 0.5 * dt_max(order, (h, h), v)
    nt = 420
    def run(n, nbl, off):
        p = Problem((n, n), (h, h), order, nbl, dt, nt, [[off + 300, off + 400]], [[off + 50, off + 400]],
                    damp_power=2, damp_vref=v)
        return Operator(p, np.full((n, n), 1 / v ** 2)).forward(synth.ricker(10.0, dt, nt))["traces"][:, 0]
    big = run(300, 0, 1100.0)
    return np.linalg.norm(run(81, 30, 0.0) - big) / np.linalg.norm(big)


def _dispersion_err(order=4):
    shape, h, v, modes = (16, 18, 20), (9.0, 11.0, 7.0), 2100.0, (3, 2, 5)
    dt = 0.8 * dt_max(order, h, v)
    nt = 200
    c = weights_f64(order)
    xi = [2 * math.pi * modes[a] / shape[a] for a in range(3)]
    lam = sum((-c[0] - 2 * sum(c[k] * math.cos(k * xi[a]) for k in range(1, len(c)))) / h[a] ** 2 for a in range(3))
    w = math.acos(1 - 0.5 * (v * dt) ** 2 * lam) / dt
    g = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    ph = sum(xi[a] * g[a] for a in range(3))
    p = Problem(shape, h, order, 0, dt, nt, np.zeros((0, 3)), np.zeros((0, 3)), periodic=True)
    out = Operator(p, np.full(shape, 1 / v ** 2)).forward(np.zeros((nt, 0)), state=(np.cos(ph), np.cos(ph) * math.cos(w * dt)))
    return np.max(np.abs(out["u"] - np.cos(ph) * math.cos(w * (nt - 1) * dt)))


def test_unmutated_baselines():
    assert _green_err_2d() < 1e-2
    assert _dot_rel() < 1e-13
    assert _grad_rel() < 1e-6
    assert _absorb_err() < 0.05
    assert _dispersion_err() < 1e-10


def test_dropped_cell_volume_in_injection(monkeypatch):
    monkeypatch.setattr(oracle.wave, "cell_volume", lambda spacing: 1.0)
    assert _green_err_2d() > 0.5


def test_source_one_step_late(monkeypatch):
    orig = Operator.step
    def late(self, u, u_prev, q_n=None):
        if q_n is not None:
            self._q_hist = getattr(self, "_q_hist", [])
            self._q_hist.append(q_n)
            q_n = self._q_hist[-2] if len(self._q_hist) > 1 else np.zeros_like(q_n)
        return orig(self, u, u_prev, q_n)
    monkeypatch.setattr(Operator, "step", late)
    assert _green_err_2d() > 1e-2


def test_damping_sign_flipped(monkeypatch):
    orig = oracle.medium.damping
    monkeypatch.setattr(oracle.wave, "damping", lambda *a, **k: -orig(*a, **k))
    assert not (_absorb_err() < 0.05)


def test_damping_dropped(monkeypatch):
    orig = oracle.medium.damping
    monkeypatch.setattr(oracle.wave, "damping", lambda *a, **k: 0.0 * orig(*a, **k))
    assert _absorb_err() > 0.05


def test_adjoint_damping_not_time_reversed(monkeypatch):
    # Using 1/B in the adjoint (damping with the wrong sense) breaks the dot test.
    def bad_adj(self, mu1, mu2, y_n=None):
        rhs = self._lap(mu1)
        if self.rec is not None and y_n is not None:
            rhs = rhs + oracle.sparse.spread(self.p.padded_shape, *self.rec, y_n)
        d_minus = self.m_pad - self.eta * self.p.dt / 2
        return (2 * self.m_pad / d_minus) * mu1 - ((self.m_pad + self.eta * self.p.dt / 2) / d_minus) * mu2 \
            + (self.p.dt ** 2 / d_minus) * rhs
    monkeypatch.setattr(Operator, "adjoint_step", bad_adj)
    assert _dot_rel() > 1e-6


def test_adjoint_missing_source_normalisation(monkeypatch):
    orig = Operator.adjoint
    def bad(self, *a, **k):
        out = orig(self, *a, **k)
        out["src_adj"] = out["src_adj"] * self.vol
        return out
    monkeypatch.setattr(Operator, "adjoint", bad)
    assert _dot_rel() > 1e-6


def test_laplacian_spacings_swapped(monkeypatch):
    orig = oracle.fd.laplacian
    monkeypatch.setattr(oracle.wave, "laplacian", lambda u, spacing, order, periodic=False:
                        orig(u, tuple(reversed(spacing)), order, periodic))
    assert _dispersion_err() > 1e-6


def test_laplacian_wrong_weight_index(monkeypatch):
    orig_w = oracle.fd.weights_f64
    def shifted(order):
        c = orig_w(order).copy()
        c[1], c[2] = c[2], c[1]
        return c
    monkeypatch.setattr(oracle.fd, "weights_f64", shifted)
    assert _dispersion_err() > 1e-6


def test_gradient_sign_flipped(monkeypatch):
    orig = Operator.adjoint
    def bad(self, *a, **k):
        out = orig(self, *a, **k)
        if "grad_pad" in out:
            out["grad_pad"] = -out["grad_pad"]
        return out
    monkeypatch.setattr(Operator, "adjoint", bad)
    assert _grad_rel() > 1.0


def test_gradient_without_padding_fold(monkeypatch):
    monkeypatch.setattr(oracle.wave, "fold_padding", lambda g, nbl: g[(slice(nbl, -nbl),) * g.ndim])
    assert _grad_rel() > 1e-4


def test_interpolation_weights_swapped():
    # Weights attached to the opposite corners: the linear-field pin fails.
    def bad(*a, **k):
        nodes, w = oracle.sparse.interpolation(*a, **k)
        return nodes, w[:, ::-1].copy()
    rng = np.random.default_rng(2)
    pts = rng.random((20, 2)) * np.array([80.0, 90.0])
    nodes, w = bad(pts, (10.0, 10.0), 2, (13, 14))
    g = np.meshgrid((np.arange(13) - 2) * 10.0, (np.arange(14) - 2) * 10.0, indexing="ij")
    f = 1.0 + 0.3 * g[0] - 0.7 * g[1]
    exact = 1.0 + 0.3 * pts[:, 0] - 0.7 * pts[:, 1]
    assert np.max(np.abs(oracle.sparse.sample(f, nodes, w) - exact)) > 1e-3
