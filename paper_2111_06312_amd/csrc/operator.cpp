// Products with the implicit design matrices as fused Horner passes.
//
// NE form, M = sum_{j=1..K} c_j T^j - lambda (1 1^T - A), T = D^-1 A (Eq. 3).
// With P = A Y, T^j Y = D^-1 (A D^-1)^(j-1) P, so
//     sum_j c_j T^j Y = D^-1 W_1,   W_K = c_K P,   W_j = c_j P + A D^-1 W_{j+1}.
// Storing W'_j = D^-1 W_j makes every pass a plain gather with A:
//     pass 1      : P = A Y                           (also writes W'_K = c_K D^-1 P)
//     pass j<K    : W'_j = D^-1 (c_j P + A W'_{j+1})
//     last (j=1)  : M Y = D^-1 (c_1 P + A W'_2) + lambda P - lambda 1 (1^T Y)
// K passes in total, and the lambda A Y term comes for free from P.
// Transpose, M^T = sum_j c_j (A^T D^-1)^j - lambda (1 1^T - A^T):
//     sum_j c_j (A^T D^-1)^j Y = A^T H_1,  H_K = c_K D^-1 Y,  H_j = D^-1 (c_j Y + A^T H_{j+1})
//     M^T Y = A^T (H_1 + lambda Y) - lambda 1 (1^T Y)
// again K passes; the first gathers Y with the column scale c_K / d_j.
// 1^T Y is summed in FP64 once per product.
//
// Feature form, M = [X, Ah X, ..., Ah^L X], Ah = (D+I)^-1/2 (A+I) (D+I)^-1/2 (Eq. 7):
//     M G = X G_0 + Ah (X G_1 + Ah (... + Ah X G_L))  : one GEMM X [G_0..G_L], then L passes
//     M^T Q = [X^T P_0; ...; X^T P_L], P_0 = Q, P_j = Ah^T P_{j-1} : L passes, one X^T [P] Gram
#include "operator.h"

#include "dag.h"

#include <algorithm>

namespace isvd {

namespace {

int64_t block_ld(int ncols) { return round_up(ncols, 8); }

template <typename T>
T* tmp_block(isvd_operator* op, int i, int64_t rows, int64_t ld) {
  op->tmp[i].ensure(static_cast<size_t>(rows) * ld * sizeof(T));
  return op->tmp[i].as<T>();
}

template <typename T>
SpmmPass base_pass(const isvd_operator* op, const Csr& csr, int ncols) {
  SpmmPass p;
  p.n_rows = op->n;
  p.nnz = csr.nnz;
  p.indptr = csr.indptr;
  p.indices = csr.indices;
  p.values = csr.values;
  p.ncols = ncols;
  p.heavy_threshold = csr.n_heavy > 0 ? op->heavy_threshold : 0;
  p.heavy_rows = csr.heavy.as<int32_t>();
  p.n_heavy = csr.n_heavy;
  return p;
}

template <typename T>
double* column_sums(isvd_operator* op, const T* Y, int64_t rows, int64_t ldy, int ncols, hipStream_t stream) {
  op->colsum_part.ensure(static_cast<size_t>(kColsumBlocks) * ncols * sizeof(double));
  op->svec.ensure(static_cast<size_t>(ncols) * sizeof(double));
  launch_colsum<T>(rows, ncols, Y, ldy, op->colsum_part.as<double>(), op->svec.as<double>(), stream);
  return op->svec.as<double>();
}

template <typename T>
void apply_ne(isvd_operator* op, bool transpose, const T* Y, int64_t ldy, int ncols, T* out, int64_t ldo,
              hipStream_t stream, const double* colsum_y) {
  const int K = op->K;
  const std::vector<double>& c = op->coeffs;  // c[j-1] = c_j
  const double lam = op->lambda;
  const Csr& csr = transpose ? op->bwd : op->fwd;
  const auto* dinv = op->scale<T>();
  const int64_t n = op->n;
  const int64_t ld = block_ld(ncols);
  const double* s = colsum_y ? colsum_y : column_sums<T>(op, Y, n, ldy, ncols, stream);

  if (!transpose) {
    if (K == 1) {
      SpmmPass p = base_pass<T>(op, csr, ncols);
      p.src = Y; p.ld_src = ldy;
      p.rowscale = dinv; p.a0 = lam; p.a1 = c[0];
      p.svec = s; p.e = -lam;
      p.out = out; p.ld_out = ldo;
      launch_spmm_pass<T>(p, stream);
      return;
    }
    T* P = tmp_block<T>(op, 0, n, ld);
    T* wa = tmp_block<T>(op, 1, n, ld);
    T* wb = tmp_block<T>(op, 2, n, ld);
    {
      SpmmPass p = base_pass<T>(op, csr, ncols);
      p.src = Y; p.ld_src = ldy;
      p.rowscale = dinv; p.a0 = 1.0;
      p.out = P; p.ld_out = ld;
      p.out2 = wa; p.ld_out2 = ld; p.c0 = 0.0; p.c1 = c[K - 1];
      launch_spmm_pass<T>(p, stream);
    }
    for (int j = K - 1; j >= 1; --j) {
      SpmmPass p = base_pass<T>(op, csr, ncols);
      p.src = wa; p.ld_src = ld;
      p.rowscale = dinv; p.a0 = 0.0; p.a1 = 1.0;
      p.add = P; p.ld_add = ld; p.b0 = 0.0; p.b1 = c[j - 1];
      if (j == 1) {
        p.b0 = lam;
        p.svec = s; p.e = -lam;
        p.out = out; p.ld_out = ldo;
      } else {
        p.out = wb; p.ld_out = ld;
      }
      launch_spmm_pass<T>(p, stream);
      std::swap(wa, wb);
    }
    return;
  }

  // transpose
  if (K == 1) {
    SpmmPass p = base_pass<T>(op, csr, ncols);
    p.src = Y; p.ld_src = ldy;
    p.colscale = dinv; p.cs_a = c[0]; p.cs_b = lam;
    p.a0 = 1.0;
    p.svec = s; p.e = -lam;
    p.out = out; p.ld_out = ldo;
    launch_spmm_pass<T>(p, stream);
    return;
  }
  T* ha = tmp_block<T>(op, 0, n, ld);
  T* hb = tmp_block<T>(op, 1, n, ld);
  for (int j = K - 1; j >= 1; --j) {
    SpmmPass p = base_pass<T>(op, csr, ncols);
    if (j == K - 1) {
      p.src = Y; p.ld_src = ldy;
      p.colscale = dinv; p.cs_a = c[K - 1]; p.cs_b = 0.0;
    } else {
      p.src = ha; p.ld_src = ld;
    }
    p.rowscale = dinv; p.a0 = 0.0; p.a1 = 1.0;
    p.add = Y; p.ld_add = ldy; p.b0 = (j == 1) ? lam : 0.0; p.b1 = c[j - 1];
    p.out = hb; p.ld_out = ld;
    launch_spmm_pass<T>(p, stream);
    std::swap(ha, hb);
  }
  SpmmPass p = base_pass<T>(op, csr, ncols);
  p.src = ha; p.ld_src = ld;
  p.a0 = 1.0;
  p.svec = s; p.e = -lam;
  p.out = out; p.ld_out = ldo;
  launch_spmm_pass<T>(p, stream);
}

template <typename T>
void apply_featprop(isvd_operator* op, bool transpose, const T* Y, int64_t ldy, int ncols, T* out,
                    int64_t ldo, hipStream_t stream) {
  using C = typename ComputeOf<T>::type;
  const int64_t n = op->n;
  const int d = static_cast<int>(op->d);
  const int L1 = op->L + 1;
  const int l = ncols;
  const int64_t wide = static_cast<int64_t>(L1) * l;
  const int64_t ldw = round_up(wide, 8);
  const T* X = static_cast<const T*>(op->X);
  const auto* dh = op->scale<T>();
  T* big = tmp_block<T>(op, 0, n, ldw);

  if (!transpose) {
    // side-by-side G blocks: Bm[a][j l + c] = G[j d + a][c]
    op->side_b.ensure(static_cast<size_t>(d) * wide * sizeof(C));
    C* Bm = op->side_b.as<C>();
    launch_stack_to_side<T, C>(d, L1, l, Y, ldy, Bm, wide, stream);
    if (L1 == 1) {
      launch_gemm_tall<T>(n, l, d, X, op->ldx, 0, nullptr, 0, Bm, wide, out, ldo, 1.0, 0.0,
                          GemmEpi::Store, nullptr, nullptr, stream);
      return;
    }
    launch_gemm_tall<T>(n, static_cast<int>(wide), d, X, op->ldx, 0, nullptr, 0, Bm, wide, big, ldw, 1.0,
                        0.0, GemmEpi::Store, nullptr, nullptr, stream);
    // Z_L = XG_L (slot L); Z_j = XG_j + Ah Z_{j+1}, written over slot j (last one to out)
    for (int j = op->L - 1; j >= 0; --j) {
      SpmmPass p = base_pass<T>(op, op->fwd, l);
      p.src = big + static_cast<int64_t>(j + 1) * l; p.ld_src = ldw;
      p.colscale = dh; p.cs_a = 1.0; p.cs_b = 0.0;
      p.rowscale = dh; p.a0 = 0.0; p.a1 = 1.0;
      p.add = big + static_cast<int64_t>(j) * l; p.ld_add = ldw; p.b0 = 1.0;
      if (j == 0) {
        p.out = out; p.ld_out = ldo;
      } else {
        p.out = big + static_cast<int64_t>(j) * l; p.ld_out = ldw;
      }
      launch_spmm_pass<T>(p, stream);
    }
    return;
  }
  // transpose: P_0 = Q (copied into slot 0), P_j = Ah^T P_{j-1}
  launch_convert<T, T>(n, l, Y, ldy, big, ldw, stream);
  for (int j = 1; j < L1; ++j) {
    SpmmPass p = base_pass<T>(op, op->bwd, l);
    p.src = big + static_cast<int64_t>(j - 1) * l; p.ld_src = ldw;
    p.colscale = dh; p.cs_a = 1.0; p.cs_b = 0.0;
    p.rowscale = dh; p.a0 = 0.0; p.a1 = 1.0;
    p.out = big + static_cast<int64_t>(j) * l; p.ld_out = ldw;
    launch_spmm_pass<T>(p, stream);
  }
  op->side_c.ensure(static_cast<size_t>(d) * wide * sizeof(double));
  op->gram_work.ensure(gram_workspace_doubles(n, d, static_cast<int>(wide)) * sizeof(double));
  launch_gram2<T, T>(n, d, static_cast<int>(wide), X, op->ldx, big, ldw, op->side_c.as<double>(), wide,
                     op->gram_work.as<double>(), stream);
  launch_side_to_stack<T>(d, L1, l, op->side_c.as<double>(), wide, out, ldo, stream);
}

void setup_csr(isvd_operator* op, Csr& csr, const int64_t* indptr, const int32_t* indices, const float* values,
               bool loops, hipStream_t stream) {
  if (loops) {
    build_loop_csr(op->n, indptr, indices, values, op->nnz, csr.own_ptr, csr.own_idx, csr.own_val, stream);
    csr.nnz = op->nnz + op->n;
    csr.indptr = csr.own_ptr.as<int64_t>();
    csr.indices = csr.own_idx.as<int32_t>();
    csr.values = values ? csr.own_val.as<float>() : nullptr;
  } else {
    csr.nnz = op->nnz;
    csr.indptr = indptr;
    csr.indices = indices;
    csr.values = values;
  }
  csr.n_heavy = build_heavy_rows(op->n, csr.indptr, op->heavy_threshold, csr.heavy, stream);
}

}  // namespace

namespace {
template <typename T>
void apply_full(isvd_operator* op, bool transpose, const T* Y, int64_t ldy, int ncols, T* out, int64_t ldo,
                hipStream_t stream, const double* colsum_y) {
  if (op->form == ISVD_FORM_NE) {
    apply_ne<T>(op, transpose, Y, ldy, ncols, out, ldo, stream, colsum_y);
  } else if (op->form == ISVD_FORM_FEATPROP) {
    apply_featprop<T>(op, transpose, Y, ldy, ncols, out, ldo, stream);
  } else {
    if constexpr (std::is_same<T, bf16>::value) {
      throw Error{ISVD_E_UNSUPPORTED, "symbolic operators take FP64 or FP32 blocks"};
    } else {
      dag_apply<T>(*op->dag_eval, transpose, Y, ldy, ncols, out, ldo, stream);
    }
  }
}
}  // namespace

// With a row gather, M_sub = M[rows, :]: M_sub Y is the full product's
// selected rows; M_sub^T Y = M^T Y' with Y' = Y's rows at the selected
// positions and zeros elsewhere (1^T Y' = 1^T Y, so colsum_y carries over).
template <typename T>
void apply_operator(isvd_operator* op, bool transpose, const T* Y, int64_t ldy, int ncols, T* out,
                    int64_t ldo, hipStream_t stream, const double* colsum_y) {
  if (op->nsel < 0) return apply_full<T>(op, transpose, Y, ldy, ncols, out, ldo, stream, colsum_y);
  const int64_t ldb = block_ld(ncols);
  op->sel_block.ensure(static_cast<size_t>(op->n) * ldb * sizeof(T));
  T* blk = op->sel_block.as<T>();
  if (!transpose) {
    apply_full<T>(op, false, Y, ldy, ncols, blk, ldb, stream, colsum_y);
    launch_gather_block<T>(op->nsel, ncols, op->sel_rows.as<int64_t>(), blk, ldb, out, ldo, stream);
  } else {
    launch_scatter_block<T>(op->n, ncols, op->sel_pos.as<int32_t>(), Y, ldy, blk, ldb, stream);
    apply_full<T>(op, true, blk, ldb, ncols, out, ldo, stream, colsum_y);
  }
}

void select_rows(isvd_operator* op, const int64_t* rows, int64_t nsel, hipStream_t stream) {
  if (!rows) {
    op->nsel = -1;
    op->rows = op->n;
    op->sel_rows.release();
    op->sel_pos.release();
    op->sel_block.release();
    return;
  }
  ISVD_CHECK(nsel >= 1 && nsel <= op->n, ISVD_E_INVALID, "row gather: need 1 <= nsub <= n");
  DevBuf flag;
  flag.ensure(sizeof(int));
  ISVD_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), stream));
  op->sel_rows.ensure(static_cast<size_t>(nsel) * sizeof(int64_t));
  ISVD_HIP(hipMemcpyAsync(op->sel_rows.p, rows, static_cast<size_t>(nsel) * sizeof(int64_t), hipMemcpyDeviceToDevice,
                          stream));
  op->sel_pos.ensure(static_cast<size_t>(op->n) * sizeof(int32_t));
  build_row_selection(op->n, nsel, op->sel_rows.as<int64_t>(), op->sel_pos.as<int32_t>(), flag.as<int>(), stream);
  int f = 0;
  ISVD_HIP(hipMemcpyAsync(&f, flag.p, sizeof(int), hipMemcpyDeviceToHost, stream));
  ISVD_HIP(hipStreamSynchronize(stream));
  if (f != 0) {
    op->nsel = -1;
    op->rows = op->n;
    throw Error{ISVD_E_INVALID, (f & 1) ? "row gather: index out of range" : "row gather: repeated index"};
  }
  op->nsel = nsel;
  op->rows = nsel;
}

template void apply_operator<double>(isvd_operator*, bool, const double*, int64_t, int, double*, int64_t, hipStream_t, const double*);
template void apply_operator<float>(isvd_operator*, bool, const float*, int64_t, int, float*, int64_t, hipStream_t, const double*);
template void apply_operator<bf16>(isvd_operator*, bool, const bf16*, int64_t, int, bf16*, int64_t, hipStream_t, const double*);

void create_operator(const isvd_graph* g, const isvd_design* m, isvd_precision prec, hipStream_t stream,
                     isvd_operator* op) {
  ISVD_CHECK(g && m, ISVD_E_INVALID, "null graph or design");
  ISVD_CHECK(g->n > 0 && g->nnz >= 0 && g->indptr && (g->nnz == 0 || g->indices), ISVD_E_INVALID,
             "graph: need n > 0 and CSR arrays");
  ISVD_CHECK(g->n < (int64_t(1) << 31), ISVD_E_INVALID, "graph: n must fit int32 column ids");
  ISVD_CHECK(prec == ISVD_FP64 || prec == ISVD_FP32 || prec == ISVD_BF16, ISVD_E_INVALID, "bad precision");
  const bool sym = g->symmetric != 0;
  ISVD_CHECK(sym || (g->t_indptr && (g->nnz == 0 || g->t_indices)), ISVD_E_INVALID,
             "directed graph needs the CSR of A^T (t_indptr, t_indices)");
  ISVD_CHECK(sym || ((g->values == nullptr) == (g->t_values == nullptr)), ISVD_E_INVALID,
             "values and t_values must both be given or both be NULL");
  op->form = m->form;
  op->prec = prec;
  op->n = g->n;
  op->nnz = g->nnz;
  op->symmetric = sym;
  op->stream = stream;
  if (m->form == ISVD_FORM_NE) {
    ISVD_CHECK(m->K >= 1 && m->coeffs, ISVD_E_INVALID, "NE form needs K >= 1 coefficients");
    op->K = m->K;
    op->coeffs.assign(m->coeffs, m->coeffs + m->K);
    op->lambda = m->lambda;
    op->rows = op->cols = g->n;
  } else if (m->form == ISVD_FORM_FEATPROP) {
    ISVD_CHECK(m->X && m->d >= 1 && m->L >= 0 && m->ldx >= m->d, ISVD_E_INVALID,
               "feature form needs X (n x d, ldx >= d) and L >= 0");
    ISVD_CHECK(m->d <= 4096, ISVD_E_INVALID, "feature width above 4096");
    op->X = m->X;
    op->d = m->d;
    op->ldx = m->ldx;
    op->L = m->L;
    op->rows = g->n;
    op->cols = m->d * (m->L + 1);
  } else {
    throw Error{ISVD_E_INVALID, "unknown design form"};
  }
  // A + I for NE with self-loops; the feature form always propagates with A + I.
  const bool loops = (m->form == ISVD_FORM_FEATPROP) || g->add_self_loops;
  setup_csr(op, op->fwd, g->indptr, g->indices, g->values, loops, stream);
  if (sym) {
    op->bwd.indptr = op->fwd.indptr;
    op->bwd.indices = op->fwd.indices;
    op->bwd.values = op->fwd.values;
    op->bwd.n_heavy = op->fwd.n_heavy;
    op->bwd.nnz = op->fwd.nnz;
    if (op->fwd.n_heavy > 0) {
      op->bwd.heavy.ensure(op->fwd.n_heavy * sizeof(int32_t));
      ISVD_HIP(hipMemcpyAsync(op->bwd.heavy.p, op->fwd.heavy.p, op->fwd.n_heavy * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, stream));
    }
  } else {
    setup_csr(op, op->bwd, g->t_indptr, g->t_indices, g->t_values, loops, stream);
  }
  // Degrees of the rows of the CSR in use (A or A+I): T = D^-1 A; for the
  // feature form, rowsum(A + I) = d + 1 gives (D + I)^-1/2.
  const int mode = m->form == ISVD_FORM_NE ? 0 : 1;
  op->deg.ensure(op->n * sizeof(double));
  op->scale32.ensure(op->n * sizeof(float));
  op->scale64.ensure(op->n * sizeof(double));
  build_row_scale<float>(op->n, op->fwd.indptr, op->fwd.values, mode, op->deg.as<double>(), op->scale32.as<float>(), stream);
  build_row_scale<double>(op->n, op->fwd.indptr, op->fwd.values, mode, op->deg.as<double>(), op->scale64.as<double>(), stream);
  ISVD_HIP(hipStreamSynchronize(stream));
}

}  // namespace isvd
