"""The C-ABI library loads, exports every declared symbol, and its host-only
functions agree with the oracle (no device work: these run without a GPU)."""
import ctypes as C

import numpy as np
import pytest

import oracle
import paper_1608_08658_amd as awe
from paper_1608_08658_amd import _lib


def test_library_exports_every_declared_symbol():
    names = _lib.header_symbols()
    assert len(names) >= 20
    handle = awe.lib()          # loads torch's HIP runtime first, then libawe.so
    missing = [n for n in names if not hasattr(handle, n)]
    assert not missing, missing
    # and the binding's table covers exactly the header
    assert sorted(_lib._SIGNATURES) == names


def test_version_string():
    assert awe.lib().awe_version().decode().startswith("awe ")


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12, 14, 16])
def test_fd_weights_match_oracle(order):
    ref = oracle.weights_f64(order)
    got = awe.fd_weights(order)
    assert np.allclose(got, ref, rtol=2e-15, atol=0)


@pytest.mark.parametrize("order", [0, 1, 3, 18, -2])
def test_fd_weights_reject_bad_order(order):
    out = (C.c_double * 16)()
    assert awe.lib().awe_fd_weights(order, out) == _lib.AWE_EINVAL
    assert "space_order" in _lib.last_error()


@pytest.mark.parametrize("ndim,order,h,v", [(2, 4, (10.0, 10.0), 1500.0), (3, 8, (10.0, 10.0, 10.0), 4950.0),
                                             (3, 16, (12.5, 12.5, 12.5), 5445.0), (2, 14, (7.0, 11.0), 3000.0)])
def test_dt_max_matches_oracle(ndim, order, h, v):
    assert awe.dt_max(ndim, order, h, v) == pytest.approx(oracle.dt_max(order, h, v), rel=1e-14)


def _geom(**over):
    kw = dict(shape=(40, 50), spacing=(10.0, 10.0), space_order=4, nbl=8, dt=1e-3, nt=100,
              src_coords=[[100.0, 200.0]], rec_coords=[[20.0, 0.0], [20.0, 10.0]])
    kw.update(over)
    return awe.make_geometry(**kw)


def test_footprint_grows_with_checkpoints():
    g = _geom()
    f0, f10, f50 = awe.footprint(g, 0), awe.footprint(g, 10), awe.footprint(g, 50)
    assert 0 < f0 < f10 and f0 < f50
    # K = 10: 18 stored + 9 slots + 3 working gradient fields beyond the forward
    per_field = (f10 - f0 - 100 * 4) / 30
    assert per_field >= (40 + 16) * (50 + 16) * 4


def test_footprint_counts_the_fields_of_the_forward():
    # C and the two wavefields, plus two work fields in 2-D (blocked steps)
    g2 = _geom()
    pts2 = (40 + 16) * (50 + 16)
    assert awe.footprint(g2, 0) >= 5 * 4 * pts2
    g3 = _geom(shape=(30, 40, 50), spacing=(10.0, 10.0, 10.0), src_coords=[[100.0, 100.0, 100.0]],
               rec_coords=[[50.0, 50.0, 50.0]])
    pts3 = (30 + 16) * (40 + 16) * (50 + 16)
    assert 3 * 4 * pts3 <= awe.footprint(g3, 0) < 5 * 4 * pts3 * 1.5


@pytest.mark.parametrize("bad", [
    dict(space_order=5), dict(space_order=18), dict(shape=(1, 50)), dict(spacing=(0.0, 10.0)),
    dict(dt=-1.0), dict(nt=0), dict(nbl=-1), dict(src_coords=[[-200.0, 0.0]]),
])
def test_invalid_geometry_is_rejected(bad):
    g = _geom(**bad)
    out = C.c_uint64()
    st = awe.lib().awe_footprint(C.byref(g.g), 0, C.byref(out))
    if "src_coords" in bad:
        # coordinates are checked when the plan builds its tables
        assert st == _lib.AWE_OK
    else:
        assert st == _lib.AWE_EINVAL
        assert _lib.last_error()


def test_null_arguments_are_errors_not_crashes():
    L = awe.lib()
    assert L.awe_footprint(None, 0, None) == _lib.AWE_EINVAL
    assert L.awe_plan_create(None, None) == _lib.AWE_EINVAL
    assert L.awe_set_model(None, None, None) == _lib.AWE_EINVAL
    assert L.awe_forward(None, None, None, 0, None) == _lib.AWE_EINVAL
    assert L.awe_adjoint(None, None, None, None, None) == _lib.AWE_EINVAL
    assert L.awe_plan_destroy(None) == _lib.AWE_OK
    assert L.awe_server_destroy(None) == _lib.AWE_OK
    assert L.awe_misfit(None, None, 0, None, None, None) == _lib.AWE_EINVAL


def test_null_arguments_of_the_newer_calls():
    import ctypes as C
    L = _lib.lib()
    i64 = C.c_int64()
    out = (C.c_double * 6)()
    assert L.awe_forward_id(None, C.byref(i64)) == _lib.AWE_EINVAL
    assert L.awe_adjoint_checked(None, 0, None, None, None, None) == _lib.AWE_EINVAL
    assert L.awe_plan_time_kernels(None, 1) == _lib.AWE_EINVAL
    assert L.awe_plan_kernel_times(None, out) == _lib.AWE_EINVAL
    assert L.awe_server_submit_gradient(None, None, None, None, None, 5, None, None, None, None) == _lib.AWE_EINVAL
    parts = (C.c_void_p * 1)(None)
    assert L.awe_sum_fields(None, parts, 1, 4, None) == _lib.AWE_EINVAL          # no output
    assert L.awe_sum_fields(C.c_void_p(16), parts, 1, 4, None) == _lib.AWE_EINVAL   # a NULL part
    assert L.awe_sum_fields(C.c_void_p(16), parts, 0, 4, None) == _lib.AWE_EINVAL   # no parts
    assert L.awe_sum_fields(C.c_void_p(16), parts, 65, 4, None) == _lib.AWE_EINVAL  # too many parts
    assert L.awe_step2_blocked(None, 1, 0, None) == _lib.AWE_EINVAL
