"""Plain FP64 CPU oracle for generalized random butterfly transform (RBT) solves.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP path
(no kernels, headers, tables or helpers); the two meet only on the seeded input
generators, which hold none of the method's arithmetic.

Paper: Lindquist, Luszczek, Dongarra, "Generalizing Random Butterfly Transforms
to Arbitrary Matrix Sizes" (ACM TOMS; arXiv 2312.09376).

Modules
  structure   reference size m and the butterfly/pairing structure (Sec. 3,
              Eq. 2-4, Algorithm 1); recursive builder (Lemma 2 recursion)
  coeffs      the counter-based SplitMix64 draw of the random diagonals
              (exp(r/20), r ~ U[-1,1], Sec. 6 setup)
  transform   dense butterfly factors (Eq. 2-3) and the packed O(d n^2)
              application (Eq. 1), both sides, forward and undo
  solve       GENP, triangular solves, undo-V, backward error (Eq. 7),
              iterative refinement (Sec. 5), adjoint of the solve
  lowprec     emulated FP32 / BF16 GENP for the mixed-precision path
  pivoted     partial-pivoting elimination and solve (the robust re-solve of
              the Sec. 5 fallback)

Parity status per function is listed in each module header.  Every function
here is pinned by a test in tests/test_oracle_*.py against something other
than itself (paper's worked example, closed forms, exact rational arithmetic,
library routines on special cases), except where a header says
"parity unpinned".
"""
from . import structure, coeffs, transform, solve, lowprec, pivoted  # noqa: F401
