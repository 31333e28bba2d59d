"""FP64 CPU oracle for the acoustic finite-difference operator of
Kukreja et al., "Devito: automated fast finite difference computation"
(arXiv:1608.08658), Sec. V.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow and deliberately
simple NumPy statement of what the operator computes.  Only ``tests/``, the
``smoke()`` check and the CPU-baseline leg of the benchmark may import it;
the GPU library never does, and the two share no code.  Its results are
pinned by properties the mathematics fixes (``tests/test_oracle_*.py``):
exact FD weights and the paper's order-2 example, polynomial exactness,
the closed-form discrete dispersion relation, the stability bound,
convergence to analytic Green's functions, source-receiver reciprocity,
the adjoint dot-product test (Eqs. 5-6), finite-difference and Taylor tests
of the gradient (Eqs. 7-8), and checkpointed == full-storage gradients.

Modules
  fd        weights (exact rationals) and the Laplacian       Sec. IV.A
  medium    padding, damping, update coefficients, CFL          Sec. V.C, V.D
  sparse    source injection / receiver interpolation           Sec. IV
  wave      forward, adjoint, misfit, gradient, checkpointing   Sec. V.A, Eqs. 1-4
  analytic  homogeneous-medium Green's functions                (physics pin)
"""
from .fd import laplacian, second_derivative_weights, weights_f64
from .medium import coefficients, damping, dt_max, fold_padding, pad_model
from .sparse import interpolation, sample, spread
from .wave import Operator, Problem, misfit

__all__ = [
    "laplacian", "second_derivative_weights", "weights_f64",
    "coefficients", "damping", "dt_max", "fold_padding", "pad_model",
    "interpolation", "sample", "spread",
    "Operator", "Problem", "misfit",
]
