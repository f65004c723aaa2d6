"""CPU oracle for the contour-integral (CI) generalized eigensolver.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package.
The GPU library never calls it and shares no code with it; the two meet
only through the seeded input generators in ``workloads``.

Contents (each function cites the passage it follows):

* ``rng``      counter-based Gaussian block (SplitMix64 + Box-Muller).
* ``cirr``     plain FP64 CIRR: sparse complex LU at every quadrature node,
               moments, SVD orthonormalisation, dense Rayleigh-Ritz,
               residuals, keep-window selection and merge.
* ``dense``    brute-force dense eigensolver (Cholesky + cyclic Jacobi)
               for small pencils.
* ``inertia``  Sylvester-inertia eigenvalue counts.

Every function here is pinned by tests against closed forms, brute force,
invariants or counts; none is marked "parity unpinned".
"""
from . import rng, dense, inertia, cirr  # noqa: F401
from .cirr import oracle_ci_solve, residuals, quadrature  # noqa: F401
