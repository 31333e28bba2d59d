"""The C time step of the oracle equals the NumPy one bit for bit."""
import numpy as np
import pytest

import synth
from oracle import Operator, Problem, dt_max


def _problem(seed, shape, h, order, nt=60):
    rng = np.random.default_rng(seed)
    v = 1500.0 + 1000.0 * rng.random(shape)
    dt = 0.6 * dt_max(order, h, v.max())
    span = np.array([(n - 1) * hh for n, hh in zip(shape, h)])
    p = Problem(shape, h, order, 3, dt, nt, rng.random((2, len(shape))) * span,
                rng.random((5, len(shape))) * span, damp_power=2, damp_vref=1500.0)
    return p, 1.0 / v ** 2, rng


@pytest.mark.parametrize("shape,h,order", [((20, 23), (10.0, 12.0), 4), ((20, 23), (7.0, 9.0), 16),
                                           ((9, 11, 10), (10.0, 9.0, 11.0), 8), ((8, 9, 10), (5.0, 6.0, 7.0), 2)])
def test_c_step_is_bitwise_equal_to_numpy(shape, h, order):
    p, m, rng = _problem(3, shape, h, order)
    w = synth.random_traces(rng, p.nt, 2, 30.0, p.dt)
    y = synth.random_traces(rng, p.nt, 5, 30.0, p.dt)
    a, b = Operator(p, m), Operator(p, m, backend="c")
    fa, fb = a.forward(w, keep=True), b.forward(w, keep=True)
    assert np.array_equal(fa["traces"], fb["traces"])
    assert np.array_equal(fa["u"], fb["u"])
    ga = a.adjoint(y, history=fa["history"])
    gb = b.adjoint(y, history=fb["history"])
    assert np.array_equal(ga["src_adj"], gb["src_adj"])
    assert np.array_equal(ga["grad_pad"], gb["grad_pad"])
