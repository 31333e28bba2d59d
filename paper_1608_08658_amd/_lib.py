"""ctypes binding of libawe.so (include/awe.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libawe.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "awe.h")

AWE_OK, AWE_EINVAL, AWE_ENOMEM, AWE_EHIP, AWE_ESTATE, AWE_EUNSTABLE, AWE_EBUSY, AWE_ENODEV = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "AWE_OK", -1: "AWE_EINVAL", -2: "AWE_ENOMEM", -3: "AWE_EHIP", -4: "AWE_ESTATE",
                -5: "AWE_EUNSTABLE", -6: "AWE_EBUSY", -7: "AWE_ENODEV"}
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3


class Geometry(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32), ("space_order", C.c_int32),
        ("shape", C.c_int64 * 3), ("spacing", C.c_double * 3),
        ("nbl", C.c_int32), ("damp_power", C.c_int32),
        ("damp_R", C.c_double), ("damp_vref", C.c_double), ("dt", C.c_double),
        ("nt", C.c_int32), ("nsrc", C.c_int32), ("nrec", C.c_int32), ("reserved", C.c_int32),
        ("src_coords", C.POINTER(C.c_double)), ("rec_coords", C.POINTER(C.c_double)),
    ]


class AweError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None

_P, _I32, _I64, _D, _U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64
_SIGNATURES = {
    "awe_last_error": (C.c_char_p, []),
    "awe_version": (C.c_char_p, []),
    "awe_fd_weights": (_I32, [_I32, C.POINTER(_D)]),
    "awe_dt_max": (_I32, [_I32, _I32, C.POINTER(_D), _D, C.POINTER(_D)]),
    "awe_footprint": (_I32, [C.POINTER(Geometry), _I32, C.POINTER(_U64)]),
    "awe_binomial_cost": (_I32, [_I32, _I32, C.POINTER(_I64), C.POINTER(_I32)]),
    "awe_footprint_binomial": (_I32, [C.POINTER(Geometry), _I32, C.POINTER(_U64)]),
    "awe_plan_create": (_I32, [C.POINTER(Geometry), C.POINTER(_P)]),
    "awe_plan_destroy": (_I32, [_P]),
    "awe_plan_info": (_I32, [_P, C.POINTER(_I64)]),
    "awe_plan_time_kernels": (_I32, [_P, _I32]),
    "awe_plan_kernel_times": (_I32, [_P, C.POINTER(_D)]),
    "awe_set_model": (_I32, [_P, _P, _P]),
    "awe_forward": (_I32, [_P, _P, _P, _I32, _P]),
    "awe_forward_binomial": (_I32, [_P, _P, _P, _I32, _P]),
    "awe_adjoint": (_I32, [_P, _P, _P, _P, _P]),
    "awe_forward_id": (_I32, [_P, C.POINTER(_I64)]),
    "awe_adjoint_checked": (_I32, [_P, _I64, _P, _P, _P, _P]),
    "awe_born": (_I32, [_P, _P, _P, _P, _P]),
    "awe_get_gradient_padded": (_I32, [_P, _P, _P]),
    "awe_set_state": (_I32, [_P, _P, _P, _P]),
    "awe_step": (_I32, [_P, _I32, _I32, _P, _P, _P]),
    "awe_step2_blocked": (_I32, [_P, _I32, _I32, _P]),
    "awe_get_state": (_I32, [_P, _P, _P, _P]),
    "awe_misfit": (_I32, [_P, _P, _I64, _P, C.POINTER(_D), _P]),
    "awe_misfit_noalloc": (_I32, [_P, _P, _I64, _P, _P, _P]),
    "awe_server_create": (_I32, [_D, _I32, _I32, C.POINTER(_P)]),
    "awe_server_submit": (_I32, [_P, C.POINTER(Geometry), _P, _P, _P, C.POINTER(_I64)]),
    "awe_server_submit_gradient": (_I32, [_P, C.POINTER(Geometry), _P, _P, _P, _I32, _P, _P, C.POINTER(_D),
                                          C.POINTER(_I64)]),
    "awe_sum_fields": (_I32, [_P, C.POINTER(_P), _I32, _I64, _P]),
    "awe_server_poll": (_I32, [_P, _I64, C.POINTER(_I32), C.POINTER(_D)]),
    "awe_server_wait": (_I32, [_P, _I64, _D]),
    "awe_server_stats": (_I32, [_P, C.POINTER(_I64)]),
    "awe_server_destroy": (_I32, [_P]),
}


def header_symbols() -> list[str]:
    """Every function name declared in include/awe.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(awe_[a-z0-9_]+)\s*\(", text)))


def _hip_runtimes_mapped() -> set[str]:
    try:
        with open("/proc/self/maps") as f:
            return {line.split()[-1] for line in f if "libamdhip64" in line}
    except OSError:
        return set()


def lib():
    """Load libawe.so once.  There is no fallback: a missing build is an error.

    torch is imported first so that its HIP runtime is the one libawe.so binds
    to (both carry the soname libamdhip64.so.7; loading libawe first would map
    a second runtime, whose streams and allocations torch's cannot see)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_1608_08658_amd.build`")
        import torch  # noqa: F401  (binds the process to torch's HIP runtime)
        handle = C.CDLL(LIB_PATH)
        runtimes = _hip_runtimes_mapped()
        if len(runtimes) > 1:
            raise RuntimeError(f"two HIP runtimes are mapped into this process: {sorted(runtimes)}")
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def last_error() -> str:
    return lib().awe_last_error().decode(errors="replace")


def check(status: int):
    if status != AWE_OK:
        raise AweError(status, last_error())
