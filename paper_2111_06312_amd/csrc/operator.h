// The implicit design-matrix operator: graph-derived data and the Horner
// drivers that evaluate M*Y and M^T*Y as sequences of fused sparse passes.
#pragma once

#include <memory>
#include <vector>

#include "common.h"
#include "dense.h"
#include "spmm.h"

namespace isvd {

// Graph ingest helpers (graph.hip).
void build_loop_csr(int64_t n, const int64_t* indptr, const int32_t* indices, const float* values,
                    int64_t nnz, DevBuf& out_ptr, DevBuf& out_idx, DevBuf& out_val, hipStream_t stream);
// mode 0: scale = 1/d (0 when d == 0); mode 1: scale = d^-1/2 (0 when d == 0).
template <typename C>
void build_row_scale(int64_t n, const int64_t* indptr, const float* values, int mode, double* deg, C* scale,
                     hipStream_t stream);
int64_t build_heavy_rows(int64_t n, const int64_t* indptr, int64_t threshold, DevBuf& list, hipStream_t stream);
// Implicit row gather: pos (n int32) from the selected rows (flag |= 1: an
// index out of range, |= 2: a repeated index); gather of the selected rows;
// scatter back into n rows with zeros elsewhere.
void build_row_selection(int64_t n, int64_t nsel, const int64_t* rows, int32_t* pos, int* flag, hipStream_t stream);
template <typename T>
void launch_gather_block(int64_t nsel, int ncols, const int64_t* rows, const T* src, int64_t lds, T* dst,
                         int64_t ldd, hipStream_t stream);
template <typename T>
void launch_scatter_block(int64_t n, int ncols, const int32_t* pos, const T* src, int64_t lds, T* dst, int64_t ldd,
                          hipStream_t stream);
template <typename T, typename C>
void launch_stack_to_side(int d, int L1, int l, const T* G, int64_t ldg, C* B, int64_t ldb, hipStream_t stream);
template <typename T>
void launch_side_to_stack(int d, int L1, int l, const double* Cm, int64_t ldc, T* out, int64_t ldo, hipStream_t stream);

// One CSR as used by the passes (borrowed or owned arrays) with its hub-row list.
struct Csr {
  const int64_t* indptr = nullptr;
  const int32_t* indices = nullptr;
  const float* values = nullptr;
  DevBuf own_ptr, own_idx, own_val, heavy;
  int64_t nnz = 0;
  int64_t n_heavy = 0;
};

struct DagEval;

}  // namespace isvd

struct isvd_operator {
  isvd_form form = ISVD_FORM_NE;
  isvd_precision prec = ISVD_FP32;
  int64_t n = 0, nnz = 0, rows = 0, cols = 0;
  bool symmetric = true;
  isvd::Csr fwd, bwd;             // CSR for M-side passes (A or A+I) and for M^T-side passes
  int64_t heavy_threshold = 256;
  isvd::DevBuf deg;               // FP64 row sums of the CSR actually used
  isvd::DevBuf scale32, scale64;  // D^-1 (NE) or (D+I)^-1/2 (feature form), float and double
  // NE
  int K = 0;
  std::vector<double> coeffs;
  double lambda = 0.0;
  // feature form
  const void* X = nullptr;
  int64_t d = 0, ldx = 0;
  int L = 0;
  // implicit row gather (rows = nsel < 0: none): the selected rows, their
  // positions, and an n-row block for the full product / scattered input
  int64_t nsel = -1;
  isvd::DevBuf sel_rows, sel_pos, sel_block;
  // workspace of the products
  isvd::DevBuf tmp[3];
  isvd::DevBuf colsum_part, svec, gram_work, side_c, side_b;
  std::shared_ptr<void> svd_cache;  // workspace of isvd_truncated_svd, kept between calls
  std::shared_ptr<isvd::DagEval> dag_eval;  // symbolic form: the evaluator of its root node
  hipStream_t stream = nullptr;

  template <typename T>
  const typename isvd::ComputeOf<T>::type* scale() const {
    if constexpr (sizeof(typename isvd::ComputeOf<T>::type) == 8) return scale64.as<double>();
    else return scale32.as<float>();
  }
};

namespace isvd {

// out = M Y (transpose = false) or M^T Y, blocks of storage type T with ncols columns.
// colsum_y (optional, NE form): 1^T Y in FP64 when the caller already has it.
template <typename T>
void apply_operator(isvd_operator* op, bool transpose, const T* Y, int64_t ldy, int ncols, T* out,
                    int64_t ldo, hipStream_t stream, const double* colsum_y = nullptr);

// Restricts the operator to M[rows, :] (rows: nsel distinct device indices,
// copied) or, with rows == NULL, back to M.  Synchronises the stream.
void select_rows(isvd_operator* op, const int64_t* rows, int64_t nsel, hipStream_t stream);

void create_operator(const isvd_graph* g, const isvd_design* m, isvd_precision prec, hipStream_t stream,
                     isvd_operator* op);

}  // namespace isvd
