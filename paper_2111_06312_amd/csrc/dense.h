// Dense kernels on tall-skinny blocks and on small l x l FP64 matrices.
#pragma once

#include "common.h"

namespace isvd {

// ---------------------------------------------------------------- Gram C = A^T B (FP64)

// Workspace (doubles) needed by launch_gram for an m x p result.
size_t gram_workspace_doubles(int64_t rows, int m, int p);

// C (m x p, FP64, ldc) = A^T B with A rows x m, B rows x p; `same` means B == A
// (only the upper tile triangle is computed and mirrored).  Partial sums per
// row slice are reduced in a fixed order.
template <typename T>
void launch_gram(int64_t rows, int m, int p, const T* A, int64_t lda, const T* B, int64_t ldb,
                 bool same, double* C, int64_t ldc, double* work, hipStream_t stream);

// launch_gram with a workspace of `work_doubles` doubles: as many row slices
// as the workspace holds (at most the default count); throws ISVD_E_INVALID
// when it cannot hold one slice's m x p partial result.
template <typename T>
void launch_gram_bounded(int64_t rows, int m, int p, const T* A, int64_t lda, const T* B, int64_t ldb, bool same,
                         double* C, int64_t ldc, double* work, size_t work_doubles, hipStream_t stream);

// Feature-side variant: A of type TA (features), B of type TB.
template <typename TA, typename TB>
void launch_gram2(int64_t rows, int m, int p, const TA* A, int64_t lda, const TB* B, int64_t ldb,
                  double* C, int64_t ldc, double* work, hipStream_t stream);

// ---------------------------------------------------------------- tall GEMM

enum class GemmEpi { Store = 0, ColNorm2 = 1 };

// C (M x N) = alpha * [A1 | A2] * B + beta * C   (A2 optional: K2 = 0)
// A1: M x K1 (ld lda1), A2: M x K2 (ld lda2), storage type T; B: (K1+K2) x N
// compute type (float for float/bf16 storage, double for double), ld ldb.
// With ColNorm2 nothing is stored; colnorm (N doubles) receives sum_rows C^2
// (two-stage reduction through `work`, gemm_colnorm_workspace doubles).
template <typename T>
void launch_gemm_tall(int64_t M, int N, int K1, const T* A1, int64_t lda1, int K2, const T* A2,
                      int64_t lda2, const typename ComputeOf<T>::type* B, int64_t ldb, T* C,
                      int64_t ldc, double alpha, double beta, GemmEpi epi, double* colnorm,
                      double* work, hipStream_t stream);
size_t gemm_colnorm_workspace(int64_t M, int N);

// ---------------------------------------------------------------- Cholesky / TRSM

// Padded size used for l x l factors (multiple of 16).
__host__ __device__ inline int pad16(int l) { return (l + 15) / 16 * 16; }

// Single-workgroup blocked Cholesky G = R^T R of an l x l SPD FP64 matrix.
// G: l x l row-major ldg.  Outputs (padded lp = pad16(l), row-major ld lp):
//   R64  : upper factor (lower triangle and padding set to the identity pattern)
//   Rc   : R in compute type C (for the tall solve), Dinv_c: inverses of the
//          16 x 16 diagonal tiles in compute type (lp/16 tiles, 256 entries each)
//   flag : three ints.  retry = 0: `shift` is added to the diagonal and
//          flag[0] = 1 on breakdown (pivot <= rel_tol * original diagonal or
//          not finite), else 0.  retry = 1: the repair launch, enqueued after
//          every retry = 0 launch so that no host round trip is needed: it
//          returns at once unless flag[0] is set, else factors G + s I with
//          s = shift * tr(G) and no pivot threshold (shifted Cholesky QR),
//          adds one to flag[2] and sets flag[1] if that fails as well.
template <typename C>
void launch_cholesky(int l, const double* G, int64_t ldg, double shift, double rel_tol, double* R64,
                     C* Rc, C* Dinv_c, int* flag, int retry, hipStream_t stream);

// In place Y <- Y R^-1 (rows x l block, storage T, ld), R/Dinv from launch_cholesky.
// colsum (optional, l doubles): FP64 column sums of the stored result, reduced
// in a fixed order through `work` (trsm_colsum_workspace doubles).
template <typename T>
void launch_trsm_tall(int64_t rows, int l, T* Y, int64_t ld, const typename ComputeOf<T>::type* Rc,
                      const typename ComputeOf<T>::type* Dinv, double* colsum, double* work,
                      hipStream_t stream);
inline size_t trsm_colsum_workspace(int l) { return static_cast<size_t>(1024) * l; }

// Y <- Y R^-1 with the block's rows in registers (used when l is at most
// trsm_rows_max_l(sizeof compute type)): launch_trsm_rows_pack packs
// launch_cholesky<double>'s R64 and the inverses of its diagonal tiles for the
// MFMA operands (Rf: trsm_rows_packed_elems(l) values of the compute type);
// launch_trsm_rows solves in place.  colsum as for launch_trsm_tall (work:
// trsm_rows_workspace doubles).
int trsm_rows_max_l(int esize);
size_t trsm_rows_packed_elems(int l);
inline size_t trsm_rows_workspace(int l) { return static_cast<size_t>(1024) * l; }
template <typename C>
void launch_trsm_rows_pack(int l, const double* R64, const double* Dinv64, C* Rf, hipStream_t stream);
template <typename T>
void launch_trsm_rows(int64_t rows, int l, T* Y, int64_t ld, const typename ComputeOf<T>::type* Rf, double* colsum,
                      double* work, hipStream_t stream);

// C = A * B for upper-triangular l x l FP64 matrices (padded lp, ld lp).
void launch_upper_mult(int l, const double* A, const double* B, double* C, int64_t ld,
                       hipStream_t stream);

// ---------------------------------------------------------------- small SVD

size_t jacobi_workspace_doubles(int n);
// A (n x n, FP64 row-major lda) = U diag(s) V^T; U, V n x n row-major (ld n), s descending.
// V0 (optional, n x n orthogonal, ld n, may alias V): starting rotation for the
// block-parallel path (64 < n <= 512), e.g. the previous V of a slowly changing A.
// rel_tol > 0 (block-parallel path): a column pair counts as orthogonal once
// |cos| <= rel_tol instead of n eps (singular vectors to about rel_tol).
void launch_jacobi_svd(int n, const double* A, int64_t lda, double* U, double* s, double* V,
                       double* work, int* sweeps_out, hipStream_t stream, const double* V0 = nullptr,
                       double rel_tol = 0.0);

// ---------------------------------------------------------------- misc

template <typename T>
void launch_gaussian(int64_t rows, int64_t cols, uint64_t seed, T* out, int64_t ld, hipStream_t stream);

// dst (rows x cols, type D) = src (type S), any lds.
template <typename D, typename S>
void launch_convert(int64_t rows, int64_t cols, const S* src, int64_t lds, D* dst, int64_t ldd,
                    hipStream_t stream);

// Pack the residual right operand B2 = [U_R(:, :k); -Z_R(:, :k) diag(s)] (2l x k, compute type).
template <typename C>
void launch_pack_residual_rhs(int l, int k, const double* UR, const double* ZR, const double* s,
                              int64_t ld, C* B, hipStream_t stream);

// Right-side residual norms |R_c z_i - s_i u_{R,i}|^2 for i < k (FP64, small).
void launch_small_residual(int l, int k, const double* Rc, int64_t ldr, const double* ZR,
                           const double* UR, int64_t ldu, const double* s, double* out,
                           hipStream_t stream);

}  // namespace isvd
