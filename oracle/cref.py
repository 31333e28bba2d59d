"""Loader for the C version of the oracle's time step (oracle/ref_step.c).

Test infrastructure, part of the CPU oracle.  The C step performs the same
floating-point operations in the same order as the NumPy step, so the two
agree bit for bit (pinned by tests/test_oracle_cref.py); it exists so that
long oracle runs (thousands of steps on 80^3 grids) finish in seconds.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ref_step.c")
LIB = os.path.join(HERE, "libawe_ref.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile ref_step.c with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                        SRC, "-o", tmp], check=True)
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        h = C.CDLL(LIB)
        h.awe_ref_step.restype = None
        P = C.c_void_p
        h.awe_ref_step.argtypes = [P, P, P, P, P, P, P, C.c_double, C.c_int, P, P, C.c_int]
        _lib = h
    return _lib


def _p(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def step(u, up, A, B, Cc, extra, div, spacing, weights):
    """out = A u - B up + C (L u + extra / div), the oracle's update in C."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    up = np.ascontiguousarray(up, dtype=np.float64)
    ndim = u.ndim
    m = len(weights) - 1
    coef = np.empty((ndim, 2 * m + 1))
    for a in range(ndim):
        inv_h2 = 1.0 / float(spacing[a]) ** 2
        for k in range(-m, m + 1):
            coef[a, k + m] = weights[abs(k)] * inv_h2
    n = np.array(u.shape, dtype=np.int64)
    out = np.empty_like(u)
    if extra is not None:
        extra = np.ascontiguousarray(extra, dtype=np.float64)
    lib().awe_ref_step(_p(u), _p(up), _p(out), _p(A), _p(B), _p(Cc), _p(extra), float(div), ndim, _p(n),
                       _p(coef), m)
    return out
