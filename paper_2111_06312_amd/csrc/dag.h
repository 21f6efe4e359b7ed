// Symbolic design matrices (Section 4 and the appendix on symbolic
// representation): the node store behind isvd_dag_* and the evaluator that
// multiplies a node onto a tall-skinny block.
#pragma once

#include <memory>
#include <vector>

#include "operator.h"

namespace isvd {

enum class DagKind { Sparse, Dense, Diag, Sum, Product, Transpose, Gather, Concat };

struct DagNode {
  DagKind kind = DagKind::Sparse;
  int64_t rows = 0, cols = 0;
  std::vector<int64_t> kids;
  std::vector<double> w;                 // Sum: weights
  Csr fwd, bwd;                          // Sparse: CSR of the matrix and of its transpose
  const void* X = nullptr;               // Dense: borrowed block
  int64_t ldx = 0;
  DevBuf d64, d32;                       // Diag: values as double and float
  DevBuf sel, pos;                       // Gather: selected rows, positions in the kid's rows
  int64_t nsub = 0;
};

// Block kernels of the evaluator (dag.hip).
template <typename T>
void launch_axpby(int64_t rows, int cols, double alpha, const T* X, int64_t ldx, double beta, T* Y, int64_t ldy,
                  hipStream_t stream);
template <typename T>
void launch_diag_scale(int64_t rows, int cols, const double* d, const T* X, int64_t ldx, T* Y, int64_t ldy,
                       hipStream_t stream);

// Evaluator state of one operator (a root node of a DAG).
struct DagEval;
std::shared_ptr<DagEval> make_dag_eval(const isvd_dag* dag, int64_t root, bool lazy_cache);
using DagStore = std::vector<std::unique_ptr<DagNode>>;
template <typename T>
void dag_apply(DagEval& ev, bool transpose, const T* Y, int64_t ldy, int ncols, T* out, int64_t ldo,
               hipStream_t stream);

}  // namespace isvd

// The node store is shared with the operators made from the DAG, so that an
// operator stays valid if the DAG handle is destroyed first.
struct isvd_dag {
  isvd_precision prec = ISVD_FP32;
  std::shared_ptr<std::vector<std::unique_ptr<isvd::DagNode>>> store =
      std::make_shared<std::vector<std::unique_ptr<isvd::DagNode>>>();
  std::vector<std::unique_ptr<isvd::DagNode>>& nodes = *store;
};
