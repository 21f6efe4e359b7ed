/*
 * isvd.h -- C ABI of the MI355X implicit randomized truncated SVD library.
 *
 * The library computes the rank-k SVD of a design matrix M that is never
 * formed (Algorithm 1 of Abu-El-Haija et al., "Implicit SVD for Graph
 * Representation Learning", NeurIPS 2021).  M is known only through
 * products M*G and M^T*G with tall-skinny dense blocks G (Section 4; the
 * appendix on symbolic representation: a matrix is usable once it offers
 * its shape, a product with an explicit block, and its transpose).
 *
 * Two design-matrix forms are built in:
 *   ISVD_FORM_NE       M = sum_{j=1..K} c_j T^j - lambda (1 1^T - A),  n x n
 *                      with T = D^-1 A (Section 2) and explicit weights c_j
 *                      (Eq. 3 takes an expectation over walk lengths; Fig. 1
 *                      builds the same matrix symbolically).
 *   ISVD_FORM_FEATPROP M = [X, Ahat X, Ahat^2 X, ..., Ahat^L X],  n x d(L+1)
 *                      with Ahat = (D+I)^-1/2 (A+I) (D+I)^-1/2 (Section 2, Eq. 7).
 * Any other M can be built as a symbolic DAG (isvd_dag_*, Section 4) and
 * used through the same operator entry points; on top of the SVD sit the
 * closed-form learners of Section 3 (isvd_ne_*, isvd_nc_fit).
 *
 * Conventions (all entry points):
 *  - Every array argument is DEVICE memory unless its comment says "host".
 *    The caller owns all memory it passes.  An operator borrows the graph
 *    arrays and X for its whole lifetime (they must stay valid and
 *    unchanged); it owns what it derives (degrees, scales, self-loop CSR,
 *    workspace).
 *  - Dense blocks are row-major with a leading dimension (elements between
 *    consecutive rows) >= their number of columns.  Their element type is
 *    the operator's precision: double (ISVD_FP64), float (ISVD_FP32) or
 *    bfloat16 bit patterns, uint16_t (ISVD_BF16).
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *  - Every function returns an isvd_status; on failure the outputs are
 *    undefined, the operator stays valid and isvd_last_error() describes
 *    the failure.  No C++ exception crosses this boundary.
 *  - Operators are not thread-safe: calls on one operator must not overlap.
 */
#ifndef ISVD_H
#define ISVD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ISVD_OK = 0,
  ISVD_E_INVALID = 1,       /* bad argument: shape mismatch, null pointer, k+p > min(r,c) ... */
  ISVD_E_OOM = 2,           /* device allocation failed */
  ISVD_E_HIP = 3,           /* a HIP runtime call failed */
  ISVD_E_NOT_SPD = 4,       /* Cholesky breakdown: Gram matrix not positive definite */
  ISVD_E_NOT_CONVERGED = 5, /* tolerance mode reached max_iter before the tolerance */
  ISVD_E_UNSUPPORTED = 6    /* valid request this build does not implement */
} isvd_status;

typedef enum {
  ISVD_FP64 = 0,  /* blocks and products in double */
  ISVD_FP32 = 1,  /* blocks in float, FP32 accumulation */
  ISVD_BF16 = 2   /* blocks stored as bfloat16, FP32 accumulation */
} isvd_precision;

typedef enum {
  ISVD_FORM_NE = 0,
  ISVD_FORM_FEATPROP = 1,
  ISVD_FORM_DAG = 2 /* an operator from isvd_dag_operator (not for isvd_create_operator) */
} isvd_form;

/* Sparse adjacency A (n x n) in CSR form, device memory, borrowed.
 * indptr has n+1 non-decreasing entries with indptr[0] = 0; indices holds
 * column ids in [0, n).  values == NULL means every stored entry is 1.
 * A directed graph (symmetric == 0) also passes the CSR of A^T in t_*
 * (t_values NULL iff values NULL).  add_self_loops replaces A by A + I
 * everywhere (degrees, T and the lambda term) for the NE form; the
 * feature-propagation form always adds I inside Ahat. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t* indptr;
  const int32_t* indices;
  const float* values;
  int symmetric;
  const int64_t* t_indptr;
  const int32_t* t_indices;
  const float* t_values;
  int add_self_loops;
} isvd_graph;

/* Design-matrix description.  coeffs is a HOST array of K doubles
 * (c_1..c_K), copied at creation.  X is a device n x d block in the
 * operator's precision (row-major, leading dimension ldx), borrowed. */
typedef struct {
  isvd_form form;
  int K;
  const double* coeffs;
  double lambda;
  const void* X;
  int64_t d;
  int64_t ldx;
  int L;
} isvd_design;

typedef struct isvd_operator isvd_operator;

const char* isvd_status_string(isvd_status s);
/* Message of the last failure on the calling thread ("" if none). */
const char* isvd_last_error(void);
/* Library version string (static). */
const char* isvd_version(void);

/* Build an operator for M from a graph and a design-matrix description
 * (Section 4: the implicit matrix).  Computes degrees D = diag(A 1), D^-1
 * (0 for zero-degree nodes, as in T's definition), (D+I)^-1/2 for the
 * feature form, and a CSR of A + I when self-loops are requested.  Work is
 * queued on `stream` and finished before return.
 * Errors: ISVD_E_INVALID (null pointers, n <= 0, K < 1, d < 1, L < 0,
 * non-symmetric graph without t_* arrays), ISVD_E_OOM, ISVD_E_HIP. */
isvd_status isvd_create_operator(const isvd_graph* graph, const isvd_design* design,
                                 isvd_precision precision, void* stream, isvd_operator** out);

/* Release the operator and everything it owns.  NULL is ignored. */
void isvd_destroy_operator(isvd_operator* op);

/* (rows, cols) of M: (n, n) for NE, (n, d(L+1)) for FEATPROP (host outputs). */
isvd_status isvd_operator_shape(const isvd_operator* op, int64_t* rows, int64_t* cols);

/* Implicit row gather (Section 3.2, option (ii); Section 4): restricts the
 * operator to M[rows, :] (say, the rows of the labelled nodes) without
 * forming M or the submatrix.  rows: nsub distinct device int64 indices in
 * [0, n) (copied; the caller may free its array after the call); rows ==
 * NULL restores M.  Afterwards isvd_operator_shape reports nsub rows and
 * isvd_matmul_block / isvd_truncated_svd work on M[rows, :]: the forward
 * product computes M Y and keeps the selected rows; the transpose places
 * the nsub-row block at the selected rows of an n-row zero block first
 * (workspace: one n x ncols block).  An index out of range or repeated:
 * ISVD_E_INVALID, and the operator is left unrestricted.  Synchronises the
 * stream. */
isvd_status isvd_operator_gather_rows(isvd_operator* op, const int64_t* rows, int64_t nsub, void* stream);

/* out = M * Y (transpose == 0; Y is cols x ncols, out is rows x ncols) or
 * out = M^T * Y (transpose != 0; Y is rows x ncols, out is cols x ncols)
 * -- the `dot` of the appendix's symbolic-matrix interface and of its
 * transpose `T`.  Y and out must not overlap.  Enqueued on `stream`
 * only; returns without synchronising.
 * Errors: ISVD_E_INVALID (null pointers, ncols < 1 or > 1024, ld < ncols). */
isvd_status isvd_matmul_block(isvd_operator* op, int transpose, const void* Y, int64_t ldy,
                              int64_t ncols, void* out, int64_t ldo, void* stream);

/* Parameters of isvd_truncated_svd.  l = k + p columns are carried
 * (Algorithm 1 carries 2k; here the width is the caller's).
 *  q         : power iterations in fixed mode (tol <= 0), as Algorithm 1's
 *              `iterations`.
 *  tol       : > 0 selects tolerance mode: iterate until the largest
 *              per-triplet relative residual
 *                rho = max_i sqrt(|M v_i - s_i u_i|^2 + |M^T u_i - s_i v_i|^2) / s_i
 *              is <= tol, or max_iter iterations.
 *  check_every : tolerance mode checks rho every this many iterations; 0 =
 *              adaptive (first check after iteration 2, then 4 iterations later,
 *              then where the observed geometric decay of rho predicts the
 *              tolerance, at most 48 iterations apart).
 *  seed      : Philox seed for a device-drawn Gaussian start block when omega is NULL.
 *  omega     : optional device c x l start block (operator precision, leading
 *              dimension ld_omega), used verbatim.
 *  fp32_switch_tol : BF16 operators only; when > 0 the iteration continues
 *              in FP32 once rho <= fp32_switch_tol, or once rho has fallen by
 *              less than 2% per iteration since the previous check, after at
 *              least 10 BF16 iterations (the BF16 rounding floor; BF16 alone
 *              cannot reach small residuals), or
 *              after bf16_max_iter iterations when that is > 0 (which replaces
 *              the 2% rule).  Without bf16_max_iter the FP32 phase first runs
 *              as a probe until its residual decay predicts the iterations
 *              still needed (taken 10% longer); while that prediction exceeds
 *              the FP32 iterations a BF16 stretch needs at its end (10) by 8
 *              or more, the blocks go back to BF16 for the difference (at most
 *              as many iterations as done so far) and the probe repeats (at
 *              most 3 times).  U and V are float for BF16 operators. */
typedef struct {
  int k;
  int p;
  int q;
  double tol;
  int max_iter;
  int check_every;
  uint64_t seed;
  const void* omega;
  int64_t ld_omega;
  double fp32_switch_tol;
  int bf16_max_iter;     /* BF16 operators: > 0 also ends the BF16 phase after this many iterations */
  int orth_passes;       /* 2: CholeskyQR2 in every iteration; otherwise one Cholesky pass (Algorithm 2)
                            in iterations whose bases only feed the next product, CholeskyQR2 before
                            every Rayleigh-Ritz step */
  int orth_method;       /* 0: Cholesky QR as above; 1: Householder QR in every orthonormalisation
                            (Algorithm 2's QR; one pass, orth_passes ignored; a slower baseline) */
} isvd_svd_params;

typedef struct {
  int iterations;        /* power iterations of the returned result (Algorithm 1's `iterations`) */
  int applies;           /* products with M or M^T performed */
  int bf16_iterations;   /* of those iterations, how many ran with BF16 blocks */
  int residual_checks;
  int used_fallback;     /* 1 if a Cholesky breakdown was repaired by a shifted re-factorisation */
  double residual;       /* rho of the returned triplets (tolerance mode), else -1 */
  double seconds;        /* wall time of the call */
  int ritz_steps;        /* small Rayleigh-Ritz SVDs computed */
  int jacobi_sweeps;     /* Jacobi sweeps of the last of them */
} isvd_svd_info;

/* Rank-k truncated SVD of M (Algorithm 1, with CholeskyQR2 as the
 * orthonormaliser in place of Algorithm 2's single Cholesky pass):
 * U (rows x k, leading dimension ldu), S (k doubles, descending), V (cols x k,
 * leading dimension ldv).  U and V are in the operator's precision, float for
 * BF16 operators.  Returns after the stream is synchronised.
 * Errors: ISVD_E_INVALID (k < 1, p < 0, k+p > min(rows, cols), q < 0,
 * tolerance mode with max_iter < 1), ISVD_E_NOT_SPD (breakdown that the
 * shifted retry could not repair), ISVD_E_NOT_CONVERGED (outputs then hold
 * the last iterate), ISVD_E_OOM, ISVD_E_HIP. */
isvd_status isvd_truncated_svd(isvd_operator* op, const isvd_svd_params* params, void* U,
                               int64_t ldu, double* S, void* V, int64_t ldv,
                               isvd_svd_info* info, void* stream);

/* ---------------------------------------------------------------------------
 * Building blocks of Algorithm 1, exported for callers that drive their own
 * iteration and for kernel-level tests.
 * ------------------------------------------------------------------------ */

/* rows x cols block of N(0,1) draws: Philox4x32-10 (Salmon et al., SC 2011),
 * pair g of row-major entries uses counter (g, 0) and key `seed`; two 53-bit
 * uniforms per pair, Box-Muller in FP64, rounded to `precision`.  Stands in
 * for Algorithm 1's Gaussian start block.  Enqueued only. */
isvd_status isvd_gaussian_block(int64_t rows, int64_t cols, uint64_t seed, isvd_precision precision,
                                void* out, int64_t ld, void* stream);

/* In place Q <- Y R^-1 with Y = Q R, R upper triangular with positive
 * diagonal (the orthonormalisation of Algorithm 2, right, run twice:
 * CholeskyQR2).  Gram Y^T Y and Cholesky in FP64, the apply in the block's
 * precision.  R_out: optional device l x l FP64 row-major output (the
 * product of both passes' factors).  Synchronises the stream.
 * Errors: ISVD_E_INVALID, ISVD_E_NOT_SPD (Gram not positive definite). */
isvd_status isvd_orthonormalize(int64_t rows, int64_t cols, isvd_precision precision, void* Y,
                                int64_t ldy, double* R_out, void* stream);

/* Householder QR of Y (rows x cols, in place: Y <- Q; R_out optional, as for
 * isvd_orthonormalize but R's diagonal may be negative), Algorithm 2's QR
 * orthonormaliser: unblocked, two passes over the trailing block per column
 * and per reflector, FP64 dot products.  1 <= cols <= min(rows, 1024).
 * Allocates a rows x cols block of workspace per call. */
isvd_status isvd_orthonormalize_householder(int64_t rows, int64_t cols, isvd_precision precision, void* Y,
                                            int64_t ldy, double* R_out, void* stream);

/* C = A^T B, A rows x m, B rows x p (same precision, leading dimensions lda,
 * ldb, m + p <= 2048), C m x p FP64 row-major (ldc), products formed exactly
 * and summed in FP64 in a fixed order.  Synchronises the stream.
 * The Gram matrices of Algorithm 2's Cholesky orthonormaliser. */
isvd_status isvd_gram(int64_t rows, int64_t m, int64_t p, isvd_precision precision, const void* A,
                      int64_t lda, const void* B, int64_t ldb, double* C, int64_t ldc, void* stream);

/* isvd_gram for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, result and error rules, but no allocation of any kind -- the
 * row-slice partial results live in a fixed 32 MiB device array of the
 * library (one per GPU, held until the process ends), so the number of row
 * slices is bounded by it and sums may group differently from isvd_gram
 * (FP64 rounding only).  Enqueued only, no synchronisation.  Every call on a
 * GPU shares that GPU's array: calls that overlap in time on one GPU race and
 * must be serialised by the caller (one stream, or host ordering). */
isvd_status isvd_gram_noalloc(int64_t rows, int64_t m, int64_t p, isvd_precision precision, const void* A,
                              int64_t lda, const void* B, int64_t ldb, double* C, int64_t ldc, void* stream);

/* SVD of a small n x n FP64 matrix (n <= 1024) by one-sided Jacobi:
 * A = Uo diag(s) Vo^T, s descending.  All device, row-major, leading dim n.
 * The small Rayleigh-Ritz SVD of Algorithm 1 (its svd of B).  Enqueued only. */
isvd_status isvd_small_svd(int64_t n, const double* A, double* Uo, double* s, double* Vo,
                           void* stream);

/* ---------------------------------------------------------------------------
 * Symbolic design matrices (Section 4 and the appendix on symbolic
 * representation): a DAG whose leaf nodes hold a matrix explicitly and whose
 * symbolic nodes are functions of other nodes; a product with a block walks
 * the DAG down to the leaves.  isvd_dag_operator turns any node into an
 * operator for isvd_matmul_block, isvd_truncated_svd and
 * isvd_operator_gather_rows.
 *
 * A DAG has one precision (ISVD_FP64 or ISVD_FP32): its dense leaves and
 * every block it multiplies are of that type.  Node ids are returned in
 * *id (>= 0).  Leaves borrow their device arrays (valid and unchanged while
 * the DAG or any operator made from it lives) except where copied is said.
 * Operators share the DAG's nodes: the DAG handle may be destroyed before
 * them.  Building nodes launches no GPU work except for
 * isvd_dag_diag and isvd_dag_gather_rows (copies, synchronised).
 *
 * Evaluation (isvd_matmul_block on a DAG operator): products are flattened
 * into chains of factors applied from the right (transposes pushed down to
 * the leaves, scalars collected); a diagonal beside a sparse leaf is fused
 * into its pass as a row or column scale; sums and concatenations
 * accumulate their terms.  With lazy_cache != 0 the result of every chain
 * suffix times the input block is kept for the duration of one product and
 * reused (the appendix's cache keyed by the ordered list of factors
 * multiplied onto the block), so t, t@t, t@t@t cost three passes, not six.
 * Workspace (device blocks of the product's width) is owned by the
 * operator and reused between calls.
 * ------------------------------------------------------------------------ */

typedef struct isvd_dag isvd_dag;

isvd_status isvd_dag_create(isvd_precision precision, isvd_dag** out);
/* Releases the DAG handle (NULL ignored); operators made from it keep its
 * nodes until they are destroyed. */
void isvd_dag_destroy(isvd_dag* dag);

/* Sparse leaf (rows x cols CSR, device, borrowed; values NULL = all ones).
 * Its transpose uses t_* (the CSR of the transpose, cols x rows) or, with
 * symmetric != 0 (rows == cols and the matrix equals its transpose), the
 * same arrays. */
isvd_status isvd_dag_sparse(isvd_dag* dag, int64_t rows, int64_t cols, int64_t nnz, const int64_t* indptr,
                            const int32_t* indices, const float* values, int symmetric, const int64_t* t_indptr,
                            const int32_t* t_indices, const float* t_values, int64_t* id);
/* Dense leaf: rows x cols row-major block X (ld ldx, the DAG's type,
 * borrowed), cols <= 2048.  Products: X G by an MFMA tall GEMM, X^T Q by
 * the FP64-MFMA Gram (cols + width <= 2048), rounded to the DAG's type. */
isvd_status isvd_dag_dense(isvd_dag* dag, int64_t rows, int64_t cols, const void* X, int64_t ldx, int64_t* id);
/* Diagonal leaf diag(d), d: n doubles (device, copied). */
isvd_status isvd_dag_diag(isvd_dag* dag, int64_t n, const double* d, int64_t* id);
/* sum_i w_i M_i over `count` nodes of one shape (ids, weights: host arrays;
 * weights NULL = all ones).  A scalar multiple is a one-term sum. */
isvd_status isvd_dag_sum(isvd_dag* dag, int count, const int64_t* ids, const double* weights, int64_t* id);
/* M_1 M_2 ... M_count (ids: host array; inner dimensions must agree).  A
 * power is a product of copies of one id. */
isvd_status isvd_dag_product(isvd_dag* dag, int count, const int64_t* ids, int64_t* id);
/* M^T. */
isvd_status isvd_dag_transpose(isvd_dag* dag, int64_t node, int64_t* id);
/* M[rows, :] (rows: nsub distinct device int64 indices, copied and checked,
 * synchronised; ISVD_E_INVALID for one out of range or repeated). */
isvd_status isvd_dag_gather_rows(isvd_dag* dag, int64_t node, const int64_t* rows, int64_t nsub, int64_t* id);
/* [M_1, ..., M_count] side by side (equal row counts; ids host).  The
 * transpose of a column concatenation stacks the parts' transposes. */
isvd_status isvd_dag_concat_cols(isvd_dag* dag, int count, const int64_t* ids, int64_t* id);
/* (rows, cols) of a node (host outputs). */
isvd_status isvd_dag_shape(const isvd_dag* dag, int64_t node, int64_t* rows, int64_t* cols);
/* An operator for node `root` (form ISVD_FORM_DAG); release it with
 * isvd_destroy_operator. */
isvd_status isvd_dag_operator(isvd_dag* dag, int64_t root, int lazy_cache, isvd_operator** out);

/* ---------------------------------------------------------------------------
 * Closed-form learners on a rank-k SVD (Section 3).  U (rows_u x k), V
 * (rows_v x k) and S (k, FP64) are the outputs of isvd_truncated_svd;
 * precision ISVD_FP64 (double U, V, Y) or ISVD_FP32 (float; BF16 operators
 * also return float U, V).  All pointers device, row-major.  Index arrays
 * are int64 and checked on the device: an index outside its range makes
 * the call return ISVD_E_INVALID (the outputs it touched are undefined).
 * isvd_ne_scores and isvd_nc_fit synchronise the stream before returning
 * (isvd_ne_embeddings only enqueues its kernel).  isvd_ne_scores and
 * isvd_nc_fit keep their device buffers in the library (one set per device,
 * grown on demand, held until the process ends) and run one at a time per
 * device (a host lock).
 * ------------------------------------------------------------------------ */

/* Node embeddings of Eq. 5: L = U S^(1/2) (rows_u x k, ldl), R = V S^(1/2)
 * (rows_v x k, ldr), in the precision of U and V.  L or R may be NULL. */
isvd_status isvd_ne_embeddings(int64_t rows_u, int64_t rows_v, int64_t k, isvd_precision precision,
                               const void* U, int64_t ldu, const double* S, const void* V, int64_t ldv,
                               void* L, int64_t ldl, void* R, int64_t ldr, void* stream);

/* Pair scores of Eq. 5: scores[p] = <L_i, R_j> = sum_t U[i][t] S[t] V[j][t]
 * with i = pi[p], j = pj[p] (FP64 products and sums; npairs doubles). */
isvd_status isvd_ne_scores(int64_t k, isvd_precision precision, const void* U, int64_t ldu, int64_t rows_u,
                           const double* S, const void* V, int64_t ldv, int64_t rows_v, int64_t npairs,
                           const int64_t* pi, const int64_t* pj, double* scores, void* stream);

/* Least-norm linear model of Eq. 8 (Theorem 1): W = V S^+ U^T Y, multiplied
 * right to left: U^T Y (FP64 sums of exact products, k + ny <= 2048), then
 * S^+ (1/s_t for s_t > rcond * max(S), else 0; rcond = 0 is the literal
 * rule), then V.  Y: rows_u x ny, the element type of U.  nsub >= 0:
 * row_subset holds nsub indices into [0, rows_u) (repeats allowed; NULL if
 * nsub = 0) and only those rows of U and Y are used (the labelled nodes,
 * Section 3.2 option (i)); nsub = -1: all rows, row_subset ignored.
 * W: rows_v x ny FP64 (zero when nsub = 0). */
isvd_status isvd_nc_fit(int64_t rows_u, int64_t rows_v, int64_t k, int64_t ny, isvd_precision precision,
                        const void* U, int64_t ldu, const double* S, const void* V, int64_t ldv, const void* Y,
                        int64_t ldy, const int64_t* row_subset, int64_t nsub, double rcond, double* W,
                        int64_t ldw, void* stream);

/* ---------------------------------------------------------------------------
 * Measurement of the sparse passes (the kernel that bounds every product).
 * ------------------------------------------------------------------------ */

/* on != 0: from now on every sparse pass is bracketed by a hipEvent pair on
 * its launch stream (two event records per pass, no host synchronisation; the
 * byte counts come from the host copy of the CSR sizes), and so are the
 * kernels of each learner call and the phases of each truncated SVD; the
 * records are cleared.  on == 0 stops recording. */
isvd_status isvd_profile_spmm_enable(int on);

/* Totals over the passes recorded since the last enable/read (host outputs):
 * summed event durations in ms, algorithmic bytes counting every gathered row
 * each time it is gathered (gather_bytes) and once per pass (compulsory_bytes),
 * and the number of passes.  Waits for the recorded events; clears the record. */
isvd_status isvd_profile_spmm_read(double* total_ms, double* gather_bytes, double* compulsory_bytes,
                                   int64_t* launches);

/* The same totals restricted to the passes whose blocks are stored in
 * `storage` (a BF16-storage SVD also runs FP32 passes in its finishing
 * phase).  Waits for the recorded events; keeps the record (the next
 * isvd_profile_spmm_read or enable clears it).  Errors: ISVD_E_INVALID. */
isvd_status isvd_profile_spmm_read_storage(isvd_precision storage, double* total_ms, double* gather_bytes,
                                           double* compulsory_bytes, int64_t* launches);

/* Totals of the learner calls recorded since the last enable/read (host
 * arrays of 3: [0] isvd_ne_embeddings, [1] isvd_ne_scores, [2] isvd_nc_fit
 * from its first kernel to its last): summed event durations in ms,
 * algorithmic bytes (U, V, Y rows read once per use, outputs written once,
 * indices), number of calls.  Waits for the events; clears the records. */
isvd_status isvd_profile_learners_read(double* ms, double* bytes, int64_t* launches);

/* Phases of the truncated SVDs run since the last enable/read (host arrays
 * of 5): [0] the products with M and M^T (Algorithm 1's applies), [1]
 * orthonormalisation (Gram, Cholesky, triangular solve; Algorithm 2),
 * [2] Rayleigh-Ritz (the small SVD), [3] residual checks, [4] the output
 * products U = Q Z, V = Q U.  ms[i]: summed durations between hipEvents
 * recorded on the SVD's stream before and after each occurrence; count[i]:
 * occurrences.  Time between phases (start block, storage switch, host
 * waits) is in none of them.  Waits for the events; clears the records.
 * Errors: ISVD_E_INVALID (null output). */
isvd_status isvd_profile_phases_read(double* ms, int64_t* count);

/* Peak rates of the device, for the rooflines of the kernels above (not
 * steps of the method).  Each call enqueues its kernels between a hipEvent
 * pair on `stream`, waits, and returns the elapsed time in *ms.
 *  isvd_peak_copy: `reps` streaming copies of `bytes` (a positive multiple of
 *    16; both device buffers 16-byte aligned) from src to dst; HBM rate =
 *    2 reps bytes / time.
 *  isvd_peak_read: one launch that reads the `bytes` of src `reps` times,
 *    each pass starting a third of the buffer further on (no L2 reuse between
 *    passes); a buffer larger than the L2s and smaller than the Infinity
 *    Cache gives that cache's read rate = reps bytes / time.
 *  isvd_peak_mfma: back-to-back independent MFMAs (16x16x4, FP64 or FP32 by
 *    `precision`), `iters` trips of 32 rounds of eight per wave; *flops receives the
 *    floating-point operations done.
 * Allocate a small device sink per call.  Errors: ISVD_E_INVALID, ISVD_E_HIP. */
isvd_status isvd_peak_copy(const void* src, void* dst, int64_t bytes, int reps, double* ms, void* stream);
isvd_status isvd_peak_read(const void* src, int64_t bytes, int reps, double* ms, void* stream);
isvd_status isvd_peak_mfma(isvd_precision precision, int64_t iters, double* flops, double* ms, void* stream);

/* ---------------------------------------------------------------------------
 * Learned warm start (not in the paper): a 16 -> 128 -> 128 -> k MLP with
 * GELU maps per-node structural features to the first k columns of the
 * start block; the remaining p columns stay Gaussian.
 * ------------------------------------------------------------------------ */

typedef struct isvd_warmstart isvd_warmstart;

/* n x 16 FP32 features of the column-side nodes of an NE operator:
 * log1p(d), log1p(T^j d) j=1..8, log1p((T^T)^j 1) j=1..7, each column
 * z-scored (a column with deviation <= 1e-9 (1 + |mean|) becomes 0).
 * F is device, row-major, leading dimension 16.  Synchronises. */
isvd_status isvd_ws_features(isvd_operator* op, float* F, void* stream);

/* New network with output width k; weights N(0, 1/fan_in) from Philox
 * `seed`, biases 0, Adam state zero. */
isvd_status isvd_ws_create(int k, uint64_t seed, isvd_warmstart** out);
void isvd_ws_destroy(isvd_warmstart* ws);
/* Total parameter count and its host layout: W1 (16x128), b1, W2 (128x128),
 * b2, W3 (128xk), b3, row-major, concatenated, float. */
int64_t isvd_ws_num_params(const isvd_warmstart* ws);
isvd_status isvd_ws_get_params(const isvd_warmstart* ws, float* host_out);
isvd_status isvd_ws_set_params(isvd_warmstart* ws, const float* host_in);

/* Z = MLP(F): F n x 16 (ld 16), Z n x k (ld ldz), both FP32 device. Enqueued only. */
isvd_status isvd_ws_forward(isvd_warmstart* ws, int64_t n, const float* F, float* Z, int64_t ldz,
                            void* stream);

/* Loss and parameter gradient for one graph: forward, subspace loss
 * L = tr((Z^T Z)^-1 Z^T (I - V V^T) Z) / k (the mean sin^2 of the principal
 * angles between span(Z) and span(V)) against orthonormal V (n x k, ld ldv,
 * FP32 device), backward.  grad_out: optional host array of
 * isvd_ws_num_params floats.  loss_out: host.  If lr > 0 an Adam step
 * (beta1 0.9, beta2 0.999, eps 1e-8) is applied.  ISVD_E_NOT_SPD, and no
 * parameter update, if Z^T Z is not positive definite.  Synchronises. */
isvd_status isvd_ws_train_step(isvd_warmstart* ws, int64_t n, const float* F, const float* V,
                               int64_t ldv, double lr, double* loss_out, float* grad_out,
                               void* stream);

/* Start block for isvd_truncated_svd from the network: omega (n x (k+p),
 * ld ld_omega, operator precision) = [sqrt(n) Q, Gaussian(seed) p columns]
 * with Q R = MLP(F) one Cholesky QR pass (orthonormal columns of the norm of
 * the Gaussian ones).  Falls back to an all-Gaussian block (and sets
 * *used_fallback = 1) when the network output is not finite or not of full
 * column rank.  Synchronises. */
isvd_status isvd_ws_omega(isvd_warmstart* ws, isvd_operator* op, const float* F, int p,
                          uint64_t seed, void* omega, int64_t ld_omega, int* used_fallback,
                          void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ISVD_H */
