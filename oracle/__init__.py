"""Plain FP64 CPU oracle for implicit randomized truncated SVD.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the package smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP
library (no kernels, headers, helpers or constants); both sides receive
the same seeded inputs from the `synth` package.

Everything here is SciPy CSR plus NumPy/LAPACK in float64, written to be
checked against the paper by eye:

- graph.py      : A, D, the transition matrix T = D^-1 A and the
                  symmetrically normalised A_hat (Section 2).
- operators.py  : products with the design matrices M^(NE) (Eq. 3 with
                  explicit weights, Fig. 1) and M^(NC) (Eq. 7), and with
                  their transposes, by the naive power sum; the
                  implicit row gather M[rows, :] (Section 3.2, option (ii)).
- symbolic.py   : the DAG of product functions of Section 4 and the
                  appendix (dense, sparse and diagonal leaves; sum, product,
                  scalar multiple, power, transpose, row gather, column and
                  row concatenation), evaluated as the definitions read.
- isvd.py       : Algorithm 1 (randomized SVD of an implicit matrix) with
                  Householder QR or Cholesky orthonormalisation
                  (Algorithm 2), and the per-triplet residual.
- learners.py   : the closed-form learners on the SVD: node embeddings and
                  pair scores (Eq. 5) and the least-norm model
                  W* = V S^+ U^T Y (Eq. 8, Theorem 1).
- mlp.py        : the warm-start network, its subspace loss and a
                  hand-derived backward pass.
- philox.py     : the Philox4x32-10 counter-based generator and the
                  Box-Muller transform used by the device start block.

Parity pins: every function here is checked by the `-m "not gpu"` tests
against closed forms, brute force on tiny inputs, invariants and LAPACK
special cases.  Two parts have no pin from the paper or from mathematics
("parity unpinned"): the residual definition (a reading, not a formula
from the paper) and the warm-start benefit (an empirical claim).
"""
