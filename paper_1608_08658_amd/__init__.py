"""awe: an MI355X-native engine for the acoustic finite-difference operator
of Kukreja et al., "Devito: automated fast finite difference computation"
(arXiv:1608.08658, Sec. V): forward modelling, its adjoint, the adjoint-state
FWI gradient with checkpointing, and a continuous-batching shot server.

The compute path is libawe.so (hand-written HIP for gfx950) behind the C ABI
of include/awe.h; this package only marshals arguments to it.
"""
from ._lib import AweError, header_symbols, lib
from .core import (Gradient, Plan, Server, binomial_cost, dt_max, fd_weights, footprint, make_geometry, misfit,
                   sum_fields)

__all__ = ["AweError", "Gradient", "Plan", "Server", "binomial_cost", "dt_max", "fd_weights", "footprint", "make_geometry",
           "misfit", "sum_fields", "header_symbols", "lib"]
