"""Plain FP64 CPU oracle for the ParaSLRF filter and eigensolver.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product path (the
HIP library and its Python binding) never does, and this package never imports
the product.  The two share no code: both consume the seeded inputs of
``slrf_inputs`` and nothing else.

Contents (each function cites the passage of the paper it follows):

* :mod:`oracle.filter` - the rational filter Phi of Eq. (3), the shifted
  systems of Eq. (2) solved exactly by sparse LU, and the filtered block
  U = sum_j 2 Re(w_j Y_j) of Algorithm 1 (conjugate-pole halving, Section 2).
* :mod:`oracle.gcr` - restarted, right-preconditioned GCR with classical
  Gram-Schmidt, the inner solver named in Section 3.2, with the stopping rule
  of Section 3.2 and the iteration cap It_max of Section 4.
* :mod:`oracle.eig` - Rayleigh-Ritz, the residual of Section 3.2,
  Algorithm 1 and Algorithm 2 (locking, B-orthogonalisation against locked
  vectors, warm start v/(theta - sigma), It_max), and a dense brute-force
  reference.
* :mod:`oracle.grad` - eigenvalue sensitivities x^T (dA - lambda dB) x summed
  per element.

Pins (what fixes each function independently of this code) are listed in the
module docstrings and exercised by the CPU tests.  Floating point is FP64
(complex128 for the shifted systems) throughout.
"""

from . import filter, gcr, eig, grad  # noqa: F401,A004
