"""FP64 CPU oracle for the shrink-and-expand block eigensolvers (arXiv 2409.05572).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The product path
(the HIP library and its Python binding) never calls it, and this package never
imports the product path.

The oracle is a plain, slow, readable restatement of the paper's algorithms in
numpy/scipy FP64. It deliberately uses different factorizations from the GPU
path (Householder QR instead of Cholesky-QR, LAPACK ``eigh`` instead of the
GPU's tridiagonal solver) and recomputes every ``A S`` product with a fresh
sparse product, so that agreement tests mathematics rather than shared code.

Modules:
* ``strategy`` - the ``fix`` / ``slope`` / ``slopek`` shrink-and-expand
  decisions (Algorithms 6 and 7, Section 3.2) with the warm-up rule.
* ``solvers``  - convergence measures (eqs. (conv) and (rk), Section 6.1),
  LOBPCG with soft locking and the Hetmaniuk-Lehoucq basis (Algorithm 3),
  subspace iteration (Algorithm 1, optionally with a Chebyshev filter), block
  steepest descent (Algorithm 2) and TraceMIN with its projected CG
  (Algorithm 4), all with shrink-and-expand (Algorithm 5), the three kinds of
  expansion vectors of Section 6 and, for LOBPCG and SD, a preconditioner.
* ``mixed``    - LOBPCG and subspace iteration (with the filter and the powered
  X_drop) with a low-precision phase (blocks stored in FP32 or BF16,
  Rayleigh-Ritz with the FP64 Gram matrix M = S^T S) followed by the FP64
  solver.

Pins: see ``tests/test_oracle_*.py``. Parity unpinned (no closed form, checked
only by invariants and by agreement with brute force at small sizes): the
Anderson and Chung-Lu eigenvalues, and every iteration count / shrink-expand
schedule produced on a matrix.
"""
from .strategy import SEParams, SEController  # noqa: F401
from .solvers import (  # noqa: F401
    SolveResult,
    residual_measures,
    orth,
    rayleigh_ritz,
    hl_basis,
    si_step,
    chebyshev_filter,
    lobpcg,
    steepest_descent,
    subspace_iteration,
    projected_cg,
    tracemin,
    jacobi_preconditioner,
)
from . import mixed  # noqa: F401,E402
