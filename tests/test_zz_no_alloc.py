"""awe_misfit_noalloc, the entry point that allocates nothing, called through
the C ABI: Φ and the residual equal awe_misfit's bit for bit on two calls in a
row, the second with a smaller input (the shared device scratch holds the
first call's partials when the second starts)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _call_both(a, b):
    import torch
    from paper_1608_08658_amd import _lib
    L = _lib.lib()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ta, tb = torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda")
    r1, r2 = torch.empty_like(ta), torch.empty_like(ta)
    phi_host = C.c_double()
    assert L.awe_misfit(C.c_void_p(ta.data_ptr()), C.c_void_p(tb.data_ptr()), ta.numel(),
                        C.c_void_p(r1.data_ptr()), C.byref(phi_host), s) == 0
    phi_dev = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    assert L.awe_misfit_noalloc(C.c_void_p(ta.data_ptr()), C.c_void_p(tb.data_ptr()), ta.numel(),
                                C.c_void_p(r2.data_ptr()), C.c_void_p(phi_dev.data_ptr()), s) == 0
    torch.cuda.synchronize()
    return phi_host.value, float(phi_dev.item()), r1.cpu().numpy(), r2.cpu().numpy()


def test_noalloc_misfit_matches_allocating_misfit():
    rng = np.random.default_rng(7)
    for n in (3_000_001, 40_961):          # the second call is smaller
        a = rng.standard_normal(n).astype(np.float32)
        b = rng.standard_normal(n).astype(np.float32)
        phi, phi_na, r1, r2 = _call_both(a, b)
        r64 = (a - b).astype(np.float64)
        print(f"n={n}: phi {phi!r} noalloc {phi_na!r}", flush=True)
        assert phi_na == phi
        assert np.array_equal(r1, r2)
        assert phi == pytest.approx(0.5 * float(np.sum(r64 * r64)), rel=1e-12)


def test_noalloc_misfit_rejects_bad_arguments():
    from paper_1608_08658_amd import _lib
    L = _lib.lib()
    assert L.awe_misfit_noalloc(None, None, 4, None, None, None) == _lib.AWE_EINVAL
    assert L.awe_misfit_noalloc(None, None, -1, None, C.c_void_p(16), None) == _lib.AWE_EINVAL
