"""Plain FP64 CPU oracle for randomized resolvent analysis (test infrastructure).

This package is the reference the HIP library is checked against.  It is test
infrastructure only: the test-suite, the package's smoke check and the CPU
baseline leg of the benchmark call it; the library itself never imports, links
or executes anything in here, and nothing in here imports the library.

It follows Ribeiro, Yeh & Taira, "Randomized resolvent analysis"
(arXiv:1902.01458): Algorithm 1 (randomized resolvent analysis), Section 2.2
(sketch, orthonormal basis, projection, reduced SVD, recovery of the response
modes through eq. (9)), Section 2.2.1 (power / subspace iteration) and
Section 3.4 / eq. (10) (physics-informed test matrix).  All arithmetic is
complex128 / float64 on the CPU with NumPy and SciPy library primitives (LAPACK
band LU, SuperLU, Householder QR, SVD) used as whole steps, never re-blocked.

Modules
  operator   2-D linearised viscous Burgers operator L (the stand-in for the
             paper's linearised Navier-Stokes operator of eq. (1))
  philox     counter-based Philox4x32-10 generator (Salmon et al., SC'11)
  sketch     physics-weighted complex Gaussian test matrix (Alg. 1 step 1, eq. 10)
  solver     factor-once, solve-many linear solves with M = i*omega*I - L
  resolvent  Algorithm 1 with subspace iteration
  dense      brute-force dense SVD of the resolvent (eq. 4, eq. 5) at small n
  grad       gradient of the leading gain (first-order perturbation of eq. 5)
  probe      unpivoted band-LU probe and conditioning report

Parity status: every function is pinned by `tests/test_oracle_*.py` against
closed forms, brute force, library routines or known-answer vectors; see the
module docstrings for which pin covers what.
"""
