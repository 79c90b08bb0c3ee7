"""CPU FP64 oracle for Sphynx-style spectral partitioning (arXiv 2105.00578).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, obviously correct
reference that the GPU path is checked against.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
path never does, and this package never imports the product path.  The two
share no code: only the seeded input generators in `graphgen` feed both.

Each function cites the passage of the paper it follows (section, equation or
algorithm).  Where the paper is silent or ambiguous, the reading taken is
stated in the function's docstring.

Modules
  laplacian  - degrees, Laplacian apply (Eq. 2 and its weighted form), dense
               Laplacian, graph classification, residual norm
  eigen      - number of eigenvectors (Eq. 4), dense smallest eigenpairs (the
               plain definition), Rayleigh-Ritz, LOBPCG (Algorithm 1)
  precond    - Jacobi, Chebyshev and GMRES-polynomial preconditioners
               (Section 5)
  split      - coordinate split into K parts (Algorithm 2, multi-jagged)
  quality    - cutsize (Eq. 1), part weights and imbalance (Section 3.1)
  adjoint    - derivative of eigenvalues / eigenvectors with respect to edge
               weights (dense full-basis reference and projected solve)
  refine     - greedy refinement of a K-way partition under the balance
               constraint (Sec. 7, Sec. 3.1)
  certify    - the d smallest eigenpairs of large graphs with error bounds
               (Algorithm 1 far past the solver's tolerance, guard vectors,
               quadratic residual and Davis-Kahan bounds)
  csrc/      - the oracle's Laplacian product as a plain C/OpenMP loop
               (built into liboracle.so with gcc; loaded by `_native`)

Pins: every function is checked in tests/test_oracle_*.py against closed forms,
library special cases, invariants or brute force.  No function here is
"parity unpinned".
"""
from . import laplacian, eigen, precond, split, quality, adjoint, refine, certify  # noqa: F401
