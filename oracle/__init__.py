"""Plain, slow, FP64 CPU oracle for randomized QR with column pivoting.

TEST INFRASTRUCTURE ONLY.  Nothing on the library's compute path imports,
calls or links anything in this package: only the test suite, the smoke check
of the entry-point module and the CPU-baseline leg of the benchmark use it.
It shares no code with the HIP library; the only thing both sides share is
the seeded input generator module (``workloads``), which holds none of the
method's arithmetic.  The random sketching matrix Omega is drawn on each side
from its own implementation of the published Philox4x64-10 generator.

Modules
-------
philox    Counter-based Gaussian Omega (Alg. 2 and Alg. 3 draw i.i.d. N(0,1)).
rqrcp     Alg. 1 (QRCP), Alg. 2 (RQRCP) with update formulas (1) and (2),
          frozen-pivot blocked QR, explicit Q.
srqr      Alg. 3 (spectrum-revealing swaps), exact and probed g2.
backward  Two independent reference gradients of Q1 [R11 R12] Pi^T with the
          pivots frozen, plus central finite differences.
compare   Column-by-column comparison of a factorization with the oracle's
          (each column against the scale its rounding errors live on).

Parity status: every function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` (brute force in exact rationals, LAPACK special
cases, the paper's Kahan tables and worked example, invariants); none is
"parity unpinned".
"""
from . import philox, rqrcp, srqr, backward, compare  # noqa: F401
