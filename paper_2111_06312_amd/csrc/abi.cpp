// extern "C" entry points: argument checks, exception barrier, last-error text.
#include <algorithm>
#include <map>
#include <mutex>
#include <string>

#include "dag.h"
#include "learners.h"
#include "operator.h"
#include "spmm.h"

namespace isvd {

isvd_status truncated_svd(isvd_operator* op, const isvd_svd_params* prm, void* U, int64_t ldu, double* S,
                          void* V, int64_t ldv, isvd_svd_info* info, hipStream_t stream);
template <typename T>
void orthonormalize_block(int64_t rows, int cols, T* Y, int64_t ld, double* Rout, hipStream_t stream,
                          bool householder);

template <typename T>
void gram_noalloc(int64_t rows, int m, int p, const T* A, int64_t lda, const T* B, int64_t ldb, bool same, double* C,
                  int64_t ldc, hipStream_t stream);
double peak_copy(const void* src, void* dst, int64_t bytes, int reps, hipStream_t stream);
double peak_read(const void* src, int64_t bytes, int reps, uint32_t* sink, hipStream_t stream);
int64_t peak_sink_elems();
double peak_mfma(bool fp64, int64_t iters, double* sink, double* flops, hipStream_t stream);

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

template <typename F>
isvd_status guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return ISVD_E_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return ISVD_E_INVALID;
  } catch (...) {
    g_last_error = "unknown error";
    return ISVD_E_INVALID;
  }
}

}  // namespace isvd

using namespace isvd;

extern "C" {

const char* isvd_status_string(isvd_status s) {
  switch (s) {
    case ISVD_OK: return "ok";
    case ISVD_E_INVALID: return "invalid argument";
    case ISVD_E_OOM: return "out of device memory";
    case ISVD_E_HIP: return "HIP runtime error";
    case ISVD_E_NOT_SPD: return "Cholesky breakdown (Gram matrix not positive definite)";
    case ISVD_E_NOT_CONVERGED: return "tolerance not reached";
    case ISVD_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* isvd_last_error(void) { return g_last_error.c_str(); }

const char* isvd_version(void) { return "isvd-mi355x 0.1 (gfx950)"; }

isvd_status isvd_create_operator(const isvd_graph* graph, const isvd_design* design, isvd_precision precision,
                                 void* stream, isvd_operator** out) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(out, ISVD_E_INVALID, "null output pointer");
    *out = nullptr;
    auto* op = new isvd_operator();
    try {
      create_operator(graph, design, precision, static_cast<hipStream_t>(stream), op);
    } catch (...) {
      delete op;
      throw;
    }
    *out = op;
    return ISVD_OK;
  });
}

void isvd_destroy_operator(isvd_operator* op) {
  if (!op) return;
  (void)hipDeviceSynchronize();
  delete op;
}

isvd_status isvd_operator_shape(const isvd_operator* op, int64_t* rows, int64_t* cols) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(op && rows && cols, ISVD_E_INVALID, "null argument");
    *rows = op->rows;
    *cols = op->cols;
    return ISVD_OK;
  });
}

isvd_status isvd_operator_gather_rows(isvd_operator* op, const int64_t* rows, int64_t nsub, void* stream) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(op, ISVD_E_INVALID, "null operator");
    select_rows(op, rows, nsub, static_cast<hipStream_t>(stream));
    return ISVD_OK;
  });
}

// ------------------------------------------------------------------ symbolic DAG

namespace {
using isvd::DagKind;
using isvd::DagNode;

DagNode& dag_node(const isvd_dag* dag, int64_t id) {
  ISVD_CHECK(dag && id >= 0 && id < static_cast<int64_t>(dag->nodes.size()), ISVD_E_INVALID, "dag: bad node id");
  return *dag->nodes[static_cast<size_t>(id)];
}

int64_t dag_add(isvd_dag* dag, std::unique_ptr<DagNode> n) {
  dag->nodes.push_back(std::move(n));
  return static_cast<int64_t>(dag->nodes.size() - 1);
}

void dag_borrow_csr(isvd::Csr& c, int64_t rows, int64_t nnz, const int64_t* indptr, const int32_t* indices,
                    const float* values) {
  c.indptr = indptr;
  c.indices = indices;
  c.values = values;
  c.nnz = nnz;
  c.n_heavy = build_heavy_rows(rows, indptr, 256, c.heavy, nullptr);
}
}  // namespace

isvd_status isvd_dag_create(isvd_precision precision, isvd_dag** out) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(out, ISVD_E_INVALID, "null output");
    ISVD_CHECK(precision == ISVD_FP64 || precision == ISVD_FP32, ISVD_E_INVALID,
               "symbolic matrices take FP64 or FP32 blocks");
    auto* d = new isvd_dag();
    d->prec = precision;
    *out = d;
    return ISVD_OK;
  });
}

void isvd_dag_destroy(isvd_dag* dag) {
  if (!dag) return;
  (void)hipDeviceSynchronize();
  delete dag;
}

isvd_status isvd_dag_sparse(isvd_dag* dag, int64_t rows, int64_t cols, int64_t nnz, const int64_t* indptr,
                            const int32_t* indices, const float* values, int symmetric, const int64_t* t_indptr,
                            const int32_t* t_indices, const float* t_values, int64_t* id) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(dag && id && rows >= 1 && cols >= 1 && nnz >= 0 && indptr && (nnz == 0 || indices), ISVD_E_INVALID,
               "dag sparse: need a CSR");
    ISVD_CHECK(rows < (int64_t(1) << 31) && cols < (int64_t(1) << 31), ISVD_E_INVALID,
               "dag sparse: dimensions must fit int32 ids");
    ISVD_CHECK(!symmetric || rows == cols, ISVD_E_INVALID, "dag sparse: a symmetric matrix is square");
    ISVD_CHECK(symmetric || (t_indptr && (nnz == 0 || t_indices) && ((values == nullptr) == (t_values == nullptr))),
               ISVD_E_INVALID, "dag sparse: a non-symmetric matrix needs the CSR of its transpose");
    auto n = std::make_unique<DagNode>();
    n->kind = DagKind::Sparse;
    n->rows = rows;
    n->cols = cols;
    dag_borrow_csr(n->fwd, rows, nnz, indptr, indices, values);
    if (symmetric)
      dag_borrow_csr(n->bwd, rows, nnz, indptr, indices, values);
    else
      dag_borrow_csr(n->bwd, cols, nnz, t_indptr, t_indices, t_values);
    ISVD_HIP(hipStreamSynchronize(nullptr));
    *id = dag_add(dag, std::move(n));
    return ISVD_OK;
  });
}

isvd_status isvd_dag_dense(isvd_dag* dag, int64_t rows, int64_t cols, const void* X, int64_t ldx, int64_t* id) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(dag && id && X && rows >= 1 && cols >= 1 && cols <= 2048 && ldx >= cols, ISVD_E_INVALID,
               "dag dense: need rows >= 1, 1 <= cols <= 2048, ldx >= cols");
    auto n = std::make_unique<DagNode>();
    n->kind = DagKind::Dense;
    n->rows = rows;
    n->cols = cols;
    n->X = X;
    n->ldx = ldx;
    *id = dag_add(dag, std::move(n));
    return ISVD_OK;
  });
}

isvd_status isvd_dag_diag(isvd_dag* dag, int64_t nd, const double* d, int64_t* id) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(dag && id && d && nd >= 1, ISVD_E_INVALID, "dag diag: need n >= 1 values");
    auto n = std::make_unique<DagNode>();
    n->kind = DagKind::Diag;
    n->rows = n->cols = nd;
    n->d64.ensure(static_cast<size_t>(nd) * sizeof(double));
    n->d32.ensure(static_cast<size_t>(nd) * sizeof(float));
    ISVD_HIP(hipMemcpyAsync(n->d64.p, d, static_cast<size_t>(nd) * sizeof(double), hipMemcpyDeviceToDevice, nullptr));
    launch_convert<float, double>(nd, 1, n->d64.as<double>(), 1, n->d32.as<float>(), 1, nullptr);
    ISVD_HIP(hipStreamSynchronize(nullptr));
    *id = dag_add(dag, std::move(n));
    return ISVD_OK;
  });
}

isvd_status isvd_dag_sum(isvd_dag* dag, int count, const int64_t* ids, const double* weights, int64_t* id) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(dag && id && ids && count >= 1, ISVD_E_INVALID, "dag sum: need at least one term");
    auto n = std::make_unique<DagNode>();
    n->kind = DagKind::Sum;
    const DagNode& first = dag_node(dag, ids[0]);
    n->rows = first.rows;
    n->cols = first.cols;
    for (int i = 0; i < count; ++i) {
      const DagNode& t = dag_node(dag, ids[i]);
      ISVD_CHECK(t.rows == n->rows && t.cols == n->cols, ISVD_E_INVALID, "dag sum: terms of different shapes");
      n->kids.push_back(ids[i]);
      n->w.push_back(weights ? weights[i] : 1.0);
    }
    *id = dag_add(dag, std::move(n));
    return ISVD_OK;
  });
}

isvd_status isvd_dag_product(isvd_dag* dag, int count, const int64_t* ids, int64_t* id) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(dag && id && ids && count >= 1, ISVD_E_INVALID, "dag product: need at least one factor");
    auto n = std::make_unique<DagNode>();
    n->kind = DagKind::Product;
    for (int i = 0; i < count; ++i) {
      const DagNode& f = dag_node(dag, ids[i]);
      if (i > 0) ISVD_CHECK(dag_node(dag, ids[i - 1]).cols == f.rows, ISVD_E_INVALID, "dag product: inner dimensions differ");
      n->kids.push_back(ids[i]);
    }
    n->rows = dag_node(dag, ids[0]).rows;
    n->cols = dag_node(dag, ids[count - 1]).cols;
    *id = dag_add(dag, std::move(n));
    return ISVD_OK;
  });
}

isvd_status isvd_dag_transpose(isvd_dag* dag, int64_t node, int64_t* id) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(id, ISVD_E_INVALID, "null output");
    const DagNode& k = dag_node(dag, node);
    auto n = std::make_unique<DagNode>();
    n->kind = DagKind::Transpose;
    n->rows = k.cols;
    n->cols = k.rows;
    n->kids.push_back(node);
    *id = dag_add(dag, std::move(n));
    return ISVD_OK;
  });
}

isvd_status isvd_dag_gather_rows(isvd_dag* dag, int64_t node, const int64_t* rows, int64_t nsub, int64_t* id) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(id && rows, ISVD_E_INVALID, "null argument");
    const DagNode& k = dag_node(dag, node);
    ISVD_CHECK(nsub >= 1 && nsub <= k.rows, ISVD_E_INVALID, "dag gather: need 1 <= nsub <= rows");
    auto n = std::make_unique<DagNode>();
    n->kind = DagKind::Gather;
    n->rows = nsub;
    n->cols = k.cols;
    n->nsub = nsub;
    n->kids.push_back(node);
    n->sel.ensure(static_cast<size_t>(nsub) * sizeof(int64_t));
    n->pos.ensure(static_cast<size_t>(k.rows) * sizeof(int32_t));
    DevBuf flag;
    flag.ensure(sizeof(int));
    ISVD_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), nullptr));
    ISVD_HIP(hipMemcpyAsync(n->sel.p, rows, static_cast<size_t>(nsub) * sizeof(int64_t), hipMemcpyDeviceToDevice,
                            nullptr));
    build_row_selection(k.rows, nsub, n->sel.as<int64_t>(), n->pos.as<int32_t>(), flag.as<int>(), nullptr);
    int f = 0;
    ISVD_HIP(hipMemcpyAsync(&f, flag.p, sizeof(int), hipMemcpyDeviceToHost, nullptr));
    ISVD_HIP(hipStreamSynchronize(nullptr));
    ISVD_CHECK(f == 0, ISVD_E_INVALID, (f & 1) ? "dag gather: index out of range" : "dag gather: repeated index");
    *id = dag_add(dag, std::move(n));
    return ISVD_OK;
  });
}

isvd_status isvd_dag_concat_cols(isvd_dag* dag, int count, const int64_t* ids, int64_t* id) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(dag && id && ids && count >= 1, ISVD_E_INVALID, "dag concat: need at least one part");
    auto n = std::make_unique<DagNode>();
    n->kind = DagKind::Concat;
    n->rows = dag_node(dag, ids[0]).rows;
    n->cols = 0;
    for (int i = 0; i < count; ++i) {
      const DagNode& p = dag_node(dag, ids[i]);
      ISVD_CHECK(p.rows == n->rows, ISVD_E_INVALID, "dag concat: parts of different row counts");
      n->kids.push_back(ids[i]);
      n->cols += p.cols;
    }
    *id = dag_add(dag, std::move(n));
    return ISVD_OK;
  });
}

isvd_status isvd_dag_shape(const isvd_dag* dag, int64_t node, int64_t* rows, int64_t* cols) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(rows && cols, ISVD_E_INVALID, "null output");
    const DagNode& n = dag_node(dag, node);
    *rows = n.rows;
    *cols = n.cols;
    return ISVD_OK;
  });
}

isvd_status isvd_dag_operator(isvd_dag* dag, int64_t root, int lazy_cache, isvd_operator** out) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(out, ISVD_E_INVALID, "null output");
    *out = nullptr;
    const DagNode& r = dag_node(dag, root);
    auto* op = new isvd_operator();
    op->form = ISVD_FORM_DAG;
    op->prec = dag->prec;
    op->n = r.rows;
    op->rows = r.rows;
    op->cols = r.cols;
    op->dag_eval = make_dag_eval(dag, root, lazy_cache != 0);
    *out = op;
    return ISVD_OK;
  });
}

isvd_status isvd_matmul_block(isvd_operator* op, int transpose, const void* Y, int64_t ldy, int64_t ncols,
                              void* out, int64_t ldo, void* stream) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(op && Y && out, ISVD_E_INVALID, "null argument");
    ISVD_CHECK(ncols >= 1 && ncols <= 1024, ISVD_E_INVALID, "ncols must be in [1, 1024]");
    ISVD_CHECK(ldy >= ncols && ldo >= ncols, ISVD_E_INVALID, "leading dimension smaller than ncols");
    ISVD_CHECK(Y != out, ISVD_E_INVALID, "Y and out must not overlap");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool t = transpose != 0;
    const int nc = static_cast<int>(ncols);
    switch (op->prec) {
      case ISVD_FP64:
        apply_operator<double>(op, t, static_cast<const double*>(Y), ldy, nc, static_cast<double*>(out), ldo, s);
        break;
      case ISVD_FP32:
        apply_operator<float>(op, t, static_cast<const float*>(Y), ldy, nc, static_cast<float*>(out), ldo, s);
        break;
      default:
        apply_operator<bf16>(op, t, static_cast<const bf16*>(Y), ldy, nc, static_cast<bf16*>(out), ldo, s);
        break;
    }
    return ISVD_OK;
  });
}

isvd_status isvd_truncated_svd(isvd_operator* op, const isvd_svd_params* params, void* U, int64_t ldu, double* S,
                               void* V, int64_t ldv, isvd_svd_info* info, void* stream) {
  return guarded([&]() -> isvd_status {
    return truncated_svd(op, params, U, ldu, S, V, ldv, info, static_cast<hipStream_t>(stream));
  });
}

isvd_status isvd_gaussian_block(int64_t rows, int64_t cols, uint64_t seed, isvd_precision precision, void* out,
                                int64_t ld, void* stream) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(out && rows >= 0 && cols >= 0 && ld >= cols, ISVD_E_INVALID, "bad block");
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (precision) {
      case ISVD_FP64: launch_gaussian<double>(rows, cols, seed, static_cast<double*>(out), ld, s); break;
      case ISVD_FP32: launch_gaussian<float>(rows, cols, seed, static_cast<float*>(out), ld, s); break;
      case ISVD_BF16: launch_gaussian<bf16>(rows, cols, seed, static_cast<bf16*>(out), ld, s); break;
      default: throw Error{ISVD_E_INVALID, "bad precision"};
    }
    return ISVD_OK;
  });
}

isvd_status isvd_orthonormalize(int64_t rows, int64_t cols, isvd_precision precision, void* Y, int64_t ldy,
                                double* R_out, void* stream) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(Y && cols >= 1 && cols <= 512 && rows >= cols && ldy >= cols, ISVD_E_INVALID,
               "need 1 <= cols <= min(rows, 512) and ldy >= cols");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int c = static_cast<int>(cols);
    switch (precision) {
      case ISVD_FP64: orthonormalize_block<double>(rows, c, static_cast<double*>(Y), ldy, R_out, s, false); break;
      case ISVD_FP32: orthonormalize_block<float>(rows, c, static_cast<float*>(Y), ldy, R_out, s, false); break;
      case ISVD_BF16: orthonormalize_block<bf16>(rows, c, static_cast<bf16*>(Y), ldy, R_out, s, false); break;
      default: throw Error{ISVD_E_INVALID, "bad precision"};
    }
    return ISVD_OK;
  });
}

isvd_status isvd_orthonormalize_householder(int64_t rows, int64_t cols, isvd_precision precision, void* Y,
                                            int64_t ldy, double* R_out, void* stream) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(Y && cols >= 1 && cols <= 1024 && rows >= cols && ldy >= cols, ISVD_E_INVALID,
               "need 1 <= cols <= min(rows, 1024) and ldy >= cols");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int c = static_cast<int>(cols);
    switch (precision) {
      case ISVD_FP64: orthonormalize_block<double>(rows, c, static_cast<double*>(Y), ldy, R_out, s, true); break;
      case ISVD_FP32: orthonormalize_block<float>(rows, c, static_cast<float*>(Y), ldy, R_out, s, true); break;
      case ISVD_BF16: orthonormalize_block<bf16>(rows, c, static_cast<bf16*>(Y), ldy, R_out, s, true); break;
      default: throw Error{ISVD_E_INVALID, "bad precision"};
    }
    return ISVD_OK;
  });
}

isvd_status isvd_gram(int64_t rows, int64_t m, int64_t p, isvd_precision precision, const void* A, int64_t lda,
                      const void* B, int64_t ldb, double* C, int64_t ldc, void* stream) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(A && B && C && rows >= 0 && m >= 1 && p >= 1 && m + p <= 2048, ISVD_E_INVALID,
               "bad gram arguments (need m + p <= 2048)");
    ISVD_CHECK(lda >= m && ldb >= p && ldc >= p, ISVD_E_INVALID, "leading dimension too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf work;
    work.ensure(gram_workspace_doubles(rows, static_cast<int>(m), static_cast<int>(p)) * sizeof(double));
    const bool same = (A == B) && (m == p) && (lda == ldb);
    switch (precision) {
      case ISVD_FP64:
        launch_gram<double>(rows, static_cast<int>(m), static_cast<int>(p), static_cast<const double*>(A), lda,
                            static_cast<const double*>(B), ldb, same, C, ldc, work.as<double>(), s);
        break;
      case ISVD_FP32:
        launch_gram<float>(rows, static_cast<int>(m), static_cast<int>(p), static_cast<const float*>(A), lda,
                           static_cast<const float*>(B), ldb, same, C, ldc, work.as<double>(), s);
        break;
      case ISVD_BF16:
        launch_gram<bf16>(rows, static_cast<int>(m), static_cast<int>(p), static_cast<const bf16*>(A), lda,
                          static_cast<const bf16*>(B), ldb, same, C, ldc, work.as<double>(), s);
        break;
      default: throw Error{ISVD_E_INVALID, "bad precision"};
    }
    ISVD_HIP(hipStreamSynchronize(s));  // the workspace is freed on return
    return ISVD_OK;
  });
}

isvd_status isvd_gram_noalloc(int64_t rows, int64_t m, int64_t p, isvd_precision precision, const void* A,
                              int64_t lda, const void* B, int64_t ldb, double* C, int64_t ldc, void* stream) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(A && B && C && rows >= 0 && m >= 1 && p >= 1 && m + p <= 2048, ISVD_E_INVALID,
               "bad gram arguments (need m + p <= 2048)");
    ISVD_CHECK(lda >= m && ldb >= p && ldc >= p, ISVD_E_INVALID, "leading dimension too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool same = (A == B) && (m == p) && (lda == ldb);
    const int mi = static_cast<int>(m), pi = static_cast<int>(p);
    switch (precision) {
      case ISVD_FP64:
        gram_noalloc<double>(rows, mi, pi, static_cast<const double*>(A), lda, static_cast<const double*>(B), ldb,
                             same, C, ldc, s);
        break;
      case ISVD_FP32:
        gram_noalloc<float>(rows, mi, pi, static_cast<const float*>(A), lda, static_cast<const float*>(B), ldb,
                            same, C, ldc, s);
        break;
      case ISVD_BF16:
        gram_noalloc<bf16>(rows, mi, pi, static_cast<const bf16*>(A), lda, static_cast<const bf16*>(B), ldb, same,
                           C, ldc, s);
        break;
      default: throw Error{ISVD_E_INVALID, "bad precision"};
    }
    return ISVD_OK;
  });
}

isvd_status isvd_small_svd(int64_t n, const double* A, double* Uo, double* s, double* Vo, void* stream) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(A && Uo && s && Vo && n >= 1 && n <= 1024, ISVD_E_INVALID, "bad small svd arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    DevBuf work;
    work.ensure(jacobi_workspace_doubles(static_cast<int>(n)) * sizeof(double));
    launch_jacobi_svd(static_cast<int>(n), A, n, Uo, s, Vo, work.as<double>(), nullptr, st);
    ISVD_HIP(hipStreamSynchronize(st));
    return ISVD_OK;
  });
}

namespace {
// Elements of U/V/Y for a learner call: FP64 or FP32 only.
size_t learner_esize(isvd_precision p) {
  ISVD_CHECK(p == ISVD_FP64 || p == ISVD_FP32, ISVD_E_INVALID,
             "learners take FP64 or FP32 factors (BF16 operators return FP32 U and V)");
  return p == ISVD_FP64 ? 8 : 4;
}
// Device buffers of the learner calls, one set per device, kept for the
// life of the process (never freed: a static destructor would run after the
// HIP runtime is gone).  A call holds its device's lock until it returns.
struct LearnerWork {
  std::mutex lock;
  DevBuf bad, ug, yg, tm, work;
};
LearnerWork& learner_work() {
  static std::mutex map_lock;
  static std::map<int, LearnerWork*>* per_device = new std::map<int, LearnerWork*>();
  int dev = 0;
  ISVD_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(map_lock);
  LearnerWork*& w = (*per_device)[dev];
  if (!w) w = new LearnerWork();
  return *w;
}
// Waits for the stream and turns the device index flag into an error.
void check_index_flag(const DevBuf& bad, hipStream_t s) {
  int flag = 0;
  ISVD_HIP(hipMemcpyAsync(&flag, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  ISVD_HIP(hipStreamSynchronize(s));
  ISVD_CHECK(flag == 0, ISVD_E_INVALID, "index out of range");
}
}  // namespace

isvd_status isvd_ne_embeddings(int64_t rows_u, int64_t rows_v, int64_t k, isvd_precision precision, const void* U,
                               int64_t ldu, const double* S, const void* V, int64_t ldv, void* L, int64_t ldl,
                               void* R, int64_t ldr, void* stream) {
  return guarded([&]() -> isvd_status {
    learner_esize(precision);
    ISVD_CHECK(S && k >= 1 && rows_u >= 0 && rows_v >= 0, ISVD_E_INVALID, "bad embedding arguments");
    ISVD_CHECK(!L || (U && ldu >= k && ldl >= k), ISVD_E_INVALID, "bad L/U arguments");
    ISVD_CHECK(!R || (V && ldv >= k && ldr >= k), ISVD_E_INVALID, "bad R/V arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    ISVD_CHECK(k <= 1024, ISVD_E_INVALID, "embeddings: k > 1024");
    const int kk = static_cast<int>(k);
    const int64_t n0 = L ? rows_u : 0, n1 = R ? rows_v : 0;
    auto embed = [&](auto tag) {
      using T = decltype(tag);
      launch_ne_embed<T>(kk, S, n0, static_cast<const T*>(U), ldu, static_cast<T*>(L), ldl, n1,
                         static_cast<const T*>(V), ldv, static_cast<T*>(R), ldr, s);
    };
    void* tok = spmm_profiling()
                    ? profile_begin(1, s, 2.0 * static_cast<double>(n0 + n1) * k * learner_esize(precision), 0.0)
                    : nullptr;
    if (precision == ISVD_FP64) embed(double{});
    else embed(float{});
    if (tok) profile_end(s, tok);
    return ISVD_OK;
  });
}

isvd_status isvd_ne_scores(int64_t k, isvd_precision precision, const void* U, int64_t ldu, int64_t rows_u,
                           const double* S, const void* V, int64_t ldv, int64_t rows_v, int64_t npairs,
                           const int64_t* pi, const int64_t* pj, double* scores, void* stream) {
  return guarded([&]() -> isvd_status {
    learner_esize(precision);
    ISVD_CHECK(U && V && S && k >= 1 && ldu >= k && ldv >= k && npairs >= 0 && (npairs == 0 || (pi && pj && scores)),
               ISVD_E_INVALID, "bad score arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    LearnerWork& lw = learner_work();
    std::lock_guard<std::mutex> hold(lw.lock);
    DevBuf& bad = lw.bad;
    bad.ensure(sizeof(int));
    ISVD_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
    const double es = static_cast<double>(learner_esize(precision));
    void* tok = spmm_profiling() && npairs > 0
                    ? profile_begin(2, s, static_cast<double>(npairs) * (2.0 * k * es + 24.0), 0.0)
                    : nullptr;
    if (precision == ISVD_FP64)
      launch_pair_scores<double>(static_cast<int>(k), static_cast<const double*>(U), ldu, rows_u, S,
                                 static_cast<const double*>(V), ldv, rows_v, npairs, pi, pj, scores, bad.as<int>(), s);
    else
      launch_pair_scores<float>(static_cast<int>(k), static_cast<const float*>(U), ldu, rows_u, S,
                                static_cast<const float*>(V), ldv, rows_v, npairs, pi, pj, scores, bad.as<int>(), s);
    if (tok) profile_end(s, tok);
    check_index_flag(bad, s);
    return ISVD_OK;
  });
}

isvd_status isvd_nc_fit(int64_t rows_u, int64_t rows_v, int64_t k, int64_t ny, isvd_precision precision,
                        const void* U, int64_t ldu, const double* S, const void* V, int64_t ldv, const void* Y,
                        int64_t ldy, const int64_t* row_subset, int64_t nsub, double rcond, double* W,
                        int64_t ldw, void* stream) {
  return guarded([&]() -> isvd_status {
    const size_t es = learner_esize(precision);
    ISVD_CHECK(U && V && S && Y && W && k >= 1 && k <= 1024 && ny >= 1 && k + ny <= 2048 && rows_u >= 0 &&
                   rows_v >= 0 && ldu >= k && ldv >= k && ldy >= ny && ldw >= ny && rcond >= 0.0,
               ISVD_E_INVALID, "bad nc fit arguments (k <= 1024, k + ny <= 2048)");
    ISVD_CHECK(nsub == -1 || (nsub >= 0 && (row_subset || nsub == 0)), ISVD_E_INVALID, "bad row subset");
    const bool subset = nsub >= 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int kk = static_cast<int>(k), yy = static_cast<int>(ny);
    ISVD_CHECK(!subset || nsub == 0 || rows_u >= 1, ISVD_E_INVALID, "index out of range");
    LearnerWork& lw = learner_work();
    std::lock_guard<std::mutex> hold(lw.lock);
    DevBuf &bad = lw.bad, &ug = lw.ug, &yg = lw.yg, &tm = lw.tm, &work = lw.work;
    bad.ensure(sizeof(int));
    ISVD_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
    const int64_t n = subset ? nsub : rows_u;
    tm.ensure(static_cast<size_t>(k) * ny * sizeof(double));
    work.ensure(gram_workspace_doubles(n, kk, yy) * sizeof(double));
    auto fit = [&](auto tag) {
      using T = decltype(tag);
      const T* u = static_cast<const T*>(U);
      const T* y = static_cast<const T*>(Y);
      int64_t lu = ldu, ly = ldy;
      if (subset && nsub > 0) {
        ug.ensure(static_cast<size_t>(std::max<int64_t>(nsub, 1)) * k * es);
        yg.ensure(static_cast<size_t>(std::max<int64_t>(nsub, 1)) * ny * es);
        launch_gather_rows<T>(nsub, row_subset, rows_u, kk, u, ldu, ug.as<T>(), k, yy, y, ldy, yg.as<T>(), ny,
                              bad.as<int>(), s);
        u = ug.as<T>();
        y = yg.as<T>();
        lu = k;
        ly = ny;
      }
      if (n == 0) {  // no labelled rows: U^T Y and W are zero
        if (rows_v > 0) ISVD_HIP(hipMemset2DAsync(W, ldw * sizeof(double), 0, ny * sizeof(double), rows_v, s));
        return;
      }
      launch_gram<T>(n, kk, yy, u, lu, y, ly, false, tm.as<double>(), ny, work.as<double>(), s);
      launch_nc_apply<T>(rows_v, kk, yy, static_cast<const T*>(V), ldv, S, rcond, tm.as<double>(), ny, W, ldw, s);
    };
    // algorithmic bytes: the used rows of U and Y (and their indices) once, V once, W written
    const double nb = static_cast<double>(n) * ((k + ny) * static_cast<double>(es) + (subset ? 8.0 : 0.0)) +
                      static_cast<double>(rows_v) * (k * static_cast<double>(es) + 8.0 * ny);
    void* tok = spmm_profiling() ? profile_begin(3, s, nb, 0.0) : nullptr;
    if (precision == ISVD_FP64) fit(double{});
    else fit(float{});
    if (tok) profile_end(s, tok);
    check_index_flag(bad, s);
    return ISVD_OK;
  });
}

isvd_status isvd_profile_spmm_enable(int on) {
  return guarded([&]() -> isvd_status {
    spmm_profile_enable(on != 0);
    return ISVD_OK;
  });
}

isvd_status isvd_profile_learners_read(double* ms, double* bytes, int64_t* launches) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(ms && bytes && launches, ISVD_E_INVALID, "null output");
    for (int c = 1; c <= kLearnerClasses; ++c)
      profile_read(c, ms + c - 1, bytes + c - 1, nullptr, launches + c - 1);
    return ISVD_OK;
  });
}

isvd_status isvd_profile_phases_read(double* ms, int64_t* count) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(ms && count, ISVD_E_INVALID, "null output");
    for (int i = 0; i < kPhaseCount; ++i) {
      double bytes = 0.0;
      profile_read(kPhaseFirst + i, ms + i, &bytes, nullptr, count + i);
    }
    return ISVD_OK;
  });
}

isvd_status isvd_profile_spmm_read(double* total_ms, double* gather_bytes, double* compulsory_bytes,
                                   int64_t* launches) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(total_ms && gather_bytes && compulsory_bytes && launches, ISVD_E_INVALID, "null argument");
    spmm_profile_read(total_ms, gather_bytes, compulsory_bytes, launches);
    return ISVD_OK;
  });
}

isvd_status isvd_profile_spmm_read_storage(isvd_precision storage, double* total_ms, double* gather_bytes,
                                           double* compulsory_bytes, int64_t* launches) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(total_ms && gather_bytes && compulsory_bytes && launches, ISVD_E_INVALID, "null argument");
    int eb = 0;
    switch (storage) {
      case ISVD_FP64: eb = 8; break;
      case ISVD_FP32: eb = 4; break;
      case ISVD_BF16: eb = 2; break;
      default: ISVD_CHECK(false, ISVD_E_INVALID, "unknown storage precision");
    }
    spmm_profile_read(total_ms, gather_bytes, compulsory_bytes, launches, eb, false);
    return ISVD_OK;
  });
}

isvd_status isvd_peak_copy(const void* src, void* dst, int64_t bytes, int reps, double* ms, void* stream) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(src && dst && ms, ISVD_E_INVALID, "null argument");
    ISVD_CHECK(bytes >= 16 && bytes % 16 == 0 && reps >= 1, ISVD_E_INVALID, "bytes: a positive multiple of 16");
    ISVD_CHECK((reinterpret_cast<uintptr_t>(src) & 15u) == 0 && (reinterpret_cast<uintptr_t>(dst) & 15u) == 0,
               ISVD_E_INVALID, "buffers must be 16-byte aligned");
    *ms = peak_copy(src, dst, bytes, reps, static_cast<hipStream_t>(stream));
    return ISVD_OK;
  });
}

isvd_status isvd_peak_read(const void* src, int64_t bytes, int reps, double* ms, void* stream) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(src && ms, ISVD_E_INVALID, "null argument");
    ISVD_CHECK(bytes >= 16 && bytes % 16 == 0 && reps >= 1, ISVD_E_INVALID, "bytes: a positive multiple of 16");
    ISVD_CHECK((reinterpret_cast<uintptr_t>(src) & 15u) == 0, ISVD_E_INVALID, "buffer must be 16-byte aligned");
    DevBuf sink;
    sink.ensure(static_cast<size_t>(peak_sink_elems()) * sizeof(uint32_t));
    *ms = peak_read(src, bytes, reps, sink.as<uint32_t>(), static_cast<hipStream_t>(stream));
    return ISVD_OK;
  });
}

isvd_status isvd_peak_mfma(isvd_precision precision, int64_t iters, double* flops, double* ms, void* stream) {
  return guarded([&]() -> isvd_status {
    ISVD_CHECK(flops && ms, ISVD_E_INVALID, "null argument");
    ISVD_CHECK(precision == ISVD_FP64 || precision == ISVD_FP32, ISVD_E_INVALID, "FP64 or FP32 only");
    ISVD_CHECK(iters >= 1, ISVD_E_INVALID, "iters >= 1");
    DevBuf sink;
    sink.ensure(static_cast<size_t>(peak_sink_elems()) * sizeof(double));
    *ms = peak_mfma(precision == ISVD_FP64, iters, sink.as<double>(), flops, static_cast<hipStream_t>(stream));
    return ISVD_OK;
  });
}

}  // extern "C"
