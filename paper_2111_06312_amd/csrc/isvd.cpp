// Algorithm 1 (randomized SVD of an implicit matrix) on the GPU.
//
// One iteration t:   Y = M Qc;  Qr, Rr = CholQR2(Y);  W = M^T Qr;  Qc, Rc = CholQR2(W)
// (the paper's loop body, its orthonormaliser being Algorithm 2's Cholesky
// variant applied twice).  Rayleigh-Ritz after iteration t: B = W^T =
// Rc^T Qc^T, so with Rc = U_R S Z_R^T (one-sided Jacobi, FP64) the triplets
// are U = Qr Z_R, S, V = Qc U_R -- Algorithm 1's svd(B) and Q x U, with B
// reduced to its l x l triangular factor.  Fixed mode runs q+1 iterations
// (Algorithm 1 with iterations = q).  Tolerance mode checks the triplets of
// iteration t during iteration t+1, whose first product M Qc gives M V for
// free:  |M v_i - s_i u_i| = column i of [Y | Qr] [U_R; -Z_R S].
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <type_traits>
#include <utility>
#include <vector>

#include "householder.h"
#include "operator.h"

namespace isvd {

namespace {

struct SvdState {
  int64_t r = 0, c = 0;
  int k = 0, l = 0, lp = 0;
  int64_t ld = 0;
  // blocks (storage of the current phase)
  DevBuf qc, w, qr, y;
  // small FP64 matrices (padded lp x lp, ld lp)
  DevBuf G, R1, R2, Rc, Rtmp, Rcc, cs_work, sum_c, sum_r, Dc, flag, UR, ZR, sig, jac_work, rhs, left2, right2, gram_work, cn_work, sweeps;
  DevBuf Rc64, Dc64, Xf;   // row-register triangular solve: FP64 factor outputs, packed operands
  bool householder = false;  // orthonormalise by Householder QR instead of Cholesky QR
  DevBuf hh_q, hh_work, hh_cs;
  int iterations = 0, applies = 0, bf16_iterations = 0, checks = 0, fallback = 0, ritz_steps = 0;
  int repairs_seen = 0;    // shifted factorisations counted at the last read of the Cholesky flags
  bool new_repairs = false;
  double residual = -1.0;
  bool have_ritz = false;
  bool zr_valid = false;   // ZR holds the right rotation of an earlier Ritz step of this call
  int ritz_iter = -1;
  int probe_need = -1;     // iterations to the tolerance predicted by a probing FP32 phase
  // convergence trace (ISVD_TRACE set in the environment): per-triplet
  // residuals and Ritz values of the last check, Ritz values of the one before
  std::vector<double> rho_i, sig_k, prev_sig_k;
  void reset_counters() {
    iterations = applies = bf16_iterations = checks = fallback = ritz_steps = repairs_seen = 0;
    new_repairs = false;
    residual = -1.0;
    have_ritz = false;
    zr_valid = false;
    ritz_iter = -1;
    rho_i.clear();
    sig_k.clear();
    prev_sig_k.clear();
  }
};

bool trace_on() {
  static const bool on = std::getenv("ISVD_TRACE") != nullptr;
  return on;
}

// One stderr line per residual check: iteration, phase, max and quantiles of
// the per-triplet residuals, Ritz values 1 and k, and the largest relative
// change of the k Ritz values since the previous check.
void trace_check(const SvdState& st, const char* phase, int t) {
  if (!trace_on() || st.rho_i.empty()) return;
  std::vector<double> r = st.rho_i;
  std::sort(r.begin(), r.end());
  const size_t k = r.size();
  double dsig = -1.0;
  if (st.prev_sig_k.size() == st.sig_k.size()) {
    dsig = 0.0;
    for (size_t i = 0; i < k; ++i)
      if (st.sig_k[i] > 0.0) dsig = std::max(dsig, std::fabs(st.sig_k[i] - st.prev_sig_k[i]) / st.sig_k[i]);
  }
  std::fprintf(stderr,
               "[isvd] %s t=%d rho max %.3e p50 %.3e p90 %.3e p99 %.3e | rho_1 %.3e rho_k %.3e | sig_1 %.6e sig_k %.6e "
               "| max rel dsig %.3e\n",
               phase, t, r[k - 1], r[k / 2], r[(9 * k) / 10], r[(99 * k) / 100], st.rho_i[0], st.rho_i[k - 1],
               st.sig_k[0], st.sig_k[k - 1], dsig);
}

// Cholesky flags (see launch_cholesky): zeroed once per call, read (with a
// stream synchronisation) only where the host needs them.
// Event bracket of one phase while profiling is on (null token otherwise).
void* phase_begin(Phase ph, hipStream_t stream) {
  return spmm_profiling() ? profile_begin(ph, stream, 0.0, 0.0) : nullptr;
}
void phase_end(hipStream_t stream, void* tok) {
  if (tok) profile_end(stream, tok);
}

void clear_chol_flags(SvdState& st, hipStream_t stream) {
  st.flag.ensure(4 * sizeof(int));
  ISVD_HIP(hipMemsetAsync(st.flag.p, 0, 4 * sizeof(int), stream));
}

void read_chol_flags(SvdState& st, hipStream_t stream) {
  int f[3] = {0, 0, 0};
  ISVD_HIP(hipMemcpyAsync(f, st.flag.p, sizeof(f), hipMemcpyDeviceToHost, stream));
  ISVD_HIP(hipStreamSynchronize(stream));
  ISVD_CHECK(f[1] == 0, ISVD_E_NOT_SPD, "Cholesky breakdown: Gram matrix not positive definite even with a shift");
  st.new_repairs = f[2] > st.repairs_seen;
  if (f[2] > 0) st.fallback = 1;
  st.repairs_seen = f[2];
}

// CholeskyQR2 of Y in place; Rout (optional) receives R2 R1; colsum (optional,
// l doubles) receives 1^T Q of the stored result.
// Y <- Y R^-1 for the factor just computed: forward substitution with the
// block's rows in registers (MFMA) when l allows, else the LDS-tiled version.
template <typename T>
void apply_rinv(SvdState& st, T* Y, int64_t rows, const double* R, bool rows_path, double* colsum,
                hipStream_t stream) {
  using C = typename ComputeOf<T>::type;
  const int l = st.l;
  if (colsum) st.cs_work.ensure(std::max(trsm_colsum_workspace(l), trsm_rows_workspace(l)) * sizeof(double));
  if (rows_path) {
    launch_trsm_rows_pack<C>(l, R, st.Dc64.as<double>(), st.Xf.as<C>(), stream);
    launch_trsm_rows<T>(rows, l, Y, st.ld, st.Xf.as<C>(), colsum, colsum ? st.cs_work.as<double>() : nullptr,
                        stream);
  } else {
    launch_trsm_tall<T>(rows, l, Y, st.ld, st.Rcc.as<C>(), st.Dc.as<C>(), colsum,
                        colsum ? st.cs_work.as<double>() : nullptr, stream);
  }
}

template <typename T>
void orthonormalize(SvdState& st, T* Y, int64_t rows, double* Rout, double* colsum, hipStream_t stream,
                    int npass = 2) {
  using C = typename ComputeOf<T>::type;
  const int l = st.l, lp = st.lp;
  if (st.householder) {
    // Algorithm 2's QR orthonormaliser: one Householder QR (backward stable, no second pass)
    st.hh_q.ensure(static_cast<size_t>(rows) * st.ld * sizeof(T));
    st.hh_work.ensure(householder_workspace_doubles(l) * sizeof(double));
    launch_householder_qr<T>(rows, l, Y, st.ld, st.hh_q.as<T>(), st.ld, Rout, lp, st.hh_work.as<double>(), stream);
    launch_convert<T, T>(rows, l, st.hh_q.as<T>(), st.ld, Y, st.ld, stream);
    if (colsum) {
      st.hh_cs.ensure(static_cast<size_t>(kColsumBlocks) * l * sizeof(double));
      launch_colsum<T>(rows, l, Y, st.ld, st.hh_cs.as<double>(), colsum, stream);
    }
    (void)npass;
    return;
  }
  const bool use_inv = l <= trsm_rows_max_l(static_cast<int>(sizeof(C)));
  st.G.ensure(static_cast<size_t>(l) * l * sizeof(double));
  st.R1.ensure(static_cast<size_t>(lp) * lp * sizeof(double));
  st.R2.ensure(static_cast<size_t>(lp) * lp * sizeof(double));
  if (use_inv) {
    st.Rc64.ensure(static_cast<size_t>(lp) * lp * sizeof(double));
    st.Dc64.ensure(static_cast<size_t>(lp) * 16 * sizeof(double));
    st.Xf.ensure(trsm_rows_packed_elems(l) * sizeof(C));
  } else {
    st.Rcc.ensure(static_cast<size_t>(lp) * lp * sizeof(C));
    st.Dc.ensure(static_cast<size_t>(lp) * 16 * sizeof(C));
  }
  // Each factorisation is followed by its repair launch (shifted Cholesky QR,
  // Fukaya et al.: G + s I with s = 11 (m l + l (l+1)) u tr(G)), which does
  // nothing unless the first one broke down, so no pass waits for the host.
  const double shift_coeff =
      11.0 * (static_cast<double>(rows) * l + static_cast<double>(l) * (l + 1)) * 1.1102230246251565e-16;
  auto factor = [&](double* Rdst) {
    for (int retry = 0; retry < 2; ++retry) {
      const double shift = retry ? shift_coeff : 0.0, rel_tol = retry ? 0.0 : 1e-14;
      if (use_inv)
        launch_cholesky<double>(l, st.G.as<double>(), l, shift, rel_tol, Rdst, st.Rc64.as<double>(),
                                st.Dc64.as<double>(), st.flag.as<int>(), retry, stream);
      else
        launch_cholesky<C>(l, st.G.as<double>(), l, shift, rel_tol, Rdst, st.Rcc.as<C>(), st.Dc.as<C>(),
                           st.flag.as<int>(), retry, stream);
    }
  };
  if (!st.flag.p) clear_chol_flags(st, stream);
  st.gram_work.ensure(gram_workspace_doubles(rows, l, l) * sizeof(double));
  double* Rp[2] = {st.R1.as<double>(), st.R2.as<double>()};
  int done = 0;
  auto run_pass = [&](bool want_colsum) {
    const int pass = done++;
    double* Rdst = Rp[pass < 2 ? pass : 1];
    if (pass >= 2) {
      // a further pass: fold R2 into R1 first (R1 <- R2 R1)
      st.Rtmp.ensure(static_cast<size_t>(lp) * lp * sizeof(double));
      launch_upper_mult(l, st.R2.as<double>(), st.R1.as<double>(), st.Rtmp.as<double>(), lp, stream);
      ISVD_HIP(hipMemcpyAsync(st.R1.p, st.Rtmp.p, static_cast<size_t>(lp) * lp * sizeof(double),
                              hipMemcpyDeviceToDevice, stream));
    }
    launch_gram<T>(rows, l, l, Y, st.ld, Y, st.ld, true, st.G.as<double>(), l, st.gram_work.as<double>(), stream);
    factor(Rdst);
    apply_rinv<T>(st, Y, rows, Rdst, use_inv, want_colsum ? colsum : nullptr, stream);
  };
  for (int pass = 0; pass < npass; ++pass) run_pass(pass + 1 == npass);
  // A single pass only has to keep the span (its result feeds the next
  // product), which the shifted factor does; its repairs are counted at the
  // next read of the flags.  Bases that must be orthonormal (two passes) are
  // checked here: after a repair, two more passes.
  if (npass >= 2) {
    for (int round = 0;; ++round) {
      read_chol_flags(st, stream);
      if (!st.new_repairs) break;
      ISVD_CHECK(round < 2, ISVD_E_NOT_SPD, "Cholesky QR: Gram matrix still needs a shift after six passes");
      run_pass(false);
      run_pass(true);
    }
  }
  if (Rout) {
    if (done == 1) launch_convert<double, double>(lp, lp, st.R1.as<double>(), lp, Rout, lp, stream);
    else launch_upper_mult(l, st.R2.as<double>(), st.R1.as<double>(), Rout, lp, stream);
  }
}

template <typename T> constexpr double kRitzTol = 1e-10;
template <> constexpr double kRitzTol<double> = 0.0;

// rel_tol: pair-orthogonality threshold of the Jacobi sweeps (0: n eps).
// Blocks stored in FP32 or BF16 carry rounding of 1e-7 and more, so their
// Ritz vectors need no more than 1e-10.
void ritz(SvdState& st, hipStream_t stream, double rel_tol = 0.0) {
  const int l = st.l, lp = st.lp;
  st.UR.ensure(static_cast<size_t>(l) * l * sizeof(double));
  st.ZR.ensure(static_cast<size_t>(l) * l * sizeof(double));
  st.sig.ensure(static_cast<size_t>(l) * sizeof(double));
  st.jac_work.ensure(jacobi_workspace_doubles(l) * sizeof(double));
  st.sweeps.ensure(sizeof(int));
  // the bases change slowly between Rayleigh-Ritz steps, so the previous right
  // rotation Z_R nearly diagonalises the new R's columns: start the sweeps there
  launch_jacobi_svd(l, st.Rc.as<double>(), lp, st.UR.as<double>(), st.sig.as<double>(), st.ZR.as<double>(),
                    st.jac_work.as<double>(), st.sweeps.as<int>(), stream,
                    st.zr_valid ? st.ZR.as<double>() : nullptr, rel_tol);
  st.have_ritz = true;
  st.zr_valid = true;
  st.ritz_steps++;
}

// rho of the current Ritz triplets, given Y = M Qc of the next iteration.
template <typename T>
double residual(SvdState& st, const T* Y, hipStream_t stream) {
  using C = typename ComputeOf<T>::type;
  const int l = st.l, k = st.k;
  st.rhs.ensure(static_cast<size_t>(2) * l * k * sizeof(C));
  st.left2.ensure(static_cast<size_t>(k) * sizeof(double));
  st.right2.ensure(static_cast<size_t>(k) * sizeof(double));
  st.cn_work.ensure(gemm_colnorm_workspace(st.r, k) * sizeof(double));
  launch_pack_residual_rhs<C>(l, k, st.UR.as<double>(), st.ZR.as<double>(), st.sig.as<double>(), l,
                              st.rhs.as<C>(), stream);
  launch_gemm_tall<T>(st.r, k, l, Y, st.ld, l, st.qr.as<T>(), st.ld, st.rhs.as<C>(), k, nullptr, 0, 1.0, 0.0,
                      GemmEpi::ColNorm2, st.left2.as<double>(), st.cn_work.as<double>(), stream);
  launch_small_residual(l, k, st.Rc.as<double>(), st.lp, st.ZR.as<double>(), st.UR.as<double>(), l,
                        st.sig.as<double>(), st.right2.as<double>(), stream);
  std::vector<double> a(k), b(k), s(k);
  ISVD_HIP(hipMemcpyAsync(a.data(), st.left2.p, k * sizeof(double), hipMemcpyDeviceToHost, stream));
  ISVD_HIP(hipMemcpyAsync(b.data(), st.right2.p, k * sizeof(double), hipMemcpyDeviceToHost, stream));
  ISVD_HIP(hipMemcpyAsync(s.data(), st.sig.p, k * sizeof(double), hipMemcpyDeviceToHost, stream));
  read_chol_flags(st, stream);   // the one synchronisation of a checked iteration
  double rho = 0.0;
  if (trace_on()) {
    st.prev_sig_k = st.sig_k;
    st.sig_k = s;
    st.rho_i.assign(k, 0.0);
  }
  for (int i = 0; i < k; ++i) {
    const double v = s[i] > 0.0 ? std::sqrt(a[i] + b[i]) / s[i] : INFINITY;
    rho = v > rho ? v : rho;
    if (trace_on()) st.rho_i[i] = v;
  }
  st.checks++;
  return rho;
}

// U = Qr Z_R[:, :k], V = Qc U_R[:, :k] (outputs of type O), S = sig[:k].
template <typename T, typename O>
void finalize(SvdState& st, isvd_operator* op, void* U, int64_t ldu, double* S, void* V, int64_t ldv,
              hipStream_t stream) {
  using C = typename ComputeOf<T>::type;
  using CO = typename ComputeOf<O>::type;
  const int l = st.l, k = st.k;
  void* tok = phase_begin(kPhaseOutput, stream);
  DevBuf zb, ub, uo, vo;
  zb.ensure(static_cast<size_t>(l) * k * sizeof(C));
  ub.ensure(static_cast<size_t>(l) * k * sizeof(C));
  launch_convert<C, double>(l, k, st.ZR.as<double>(), l, zb.as<C>(), k, stream);
  launch_convert<C, double>(l, k, st.UR.as<double>(), l, ub.as<C>(), k, stream);
  if constexpr (std::is_same<T, O>::value) {
    launch_gemm_tall<T>(st.r, k, l, st.qr.as<T>(), st.ld, 0, nullptr, 0, zb.as<C>(), k, static_cast<T*>(U), ldu,
                        1.0, 0.0, GemmEpi::Store, nullptr, nullptr, stream);
    launch_gemm_tall<T>(st.c, k, l, st.qc.as<T>(), st.ld, 0, nullptr, 0, ub.as<C>(), k, static_cast<T*>(V), ldv,
                        1.0, 0.0, GemmEpi::Store, nullptr, nullptr, stream);
  } else {
    // BF16 blocks, float outputs: widen the blocks first (exact), then multiply in FP32.
    static_assert(std::is_same<CO, float>::value, "widening only to float");
    DevBuf wide;
    const int64_t rows = st.r > st.c ? st.r : st.c;
    wide.ensure(static_cast<size_t>(rows) * st.ld * sizeof(float));
    launch_convert<float, T>(st.r, l, st.qr.as<T>(), st.ld, wide.as<float>(), st.ld, stream);
    launch_gemm_tall<float>(st.r, k, l, wide.as<float>(), st.ld, 0, nullptr, 0, zb.as<float>(), k,
                            static_cast<float*>(U), ldu, 1.0, 0.0, GemmEpi::Store, nullptr, nullptr, stream);
    launch_convert<float, T>(st.c, l, st.qc.as<T>(), st.ld, wide.as<float>(), st.ld, stream);
    launch_gemm_tall<float>(st.c, k, l, wide.as<float>(), st.ld, 0, nullptr, 0, ub.as<float>(), k,
                            static_cast<float*>(V), ldv, 1.0, 0.0, GemmEpi::Store, nullptr, nullptr, stream);
    ISVD_HIP(hipStreamSynchronize(stream));
  }
  phase_end(stream, tok);
  ISVD_HIP(hipMemcpyAsync(S, st.sig.p, k * sizeof(double), hipMemcpyDeviceToDevice, stream));
  ISVD_HIP(hipStreamSynchronize(stream));
  (void)op;
}

template <typename T>
void ensure_blocks(SvdState& st) {
  st.qc.ensure(static_cast<size_t>(st.c) * st.ld * sizeof(T));
  st.w.ensure(static_cast<size_t>(st.c) * st.ld * sizeof(T));
  st.qr.ensure(static_cast<size_t>(st.r) * st.ld * sizeof(T));
  st.y.ensure(static_cast<size_t>(st.r) * st.ld * sizeof(T));
  st.Rc.ensure(static_cast<size_t>(st.lp) * st.lp * sizeof(double));
}

// Iteration at which the next Rayleigh-Ritz step (and residual check) runs.
// check_every > 0: a fixed stride.  check_every == 0: adaptive -- the residual
// decays about geometrically, so the rate seen between the last two checks
// predicts how many more iterations reach `tol`; the next check is placed at
// 90% of that distance (at least 1 and at most kMaxCheckGap iterations ahead).
constexpr int kFirstCheck = 2;    // iterations before the first residual check
constexpr int kStallMinIter = 10; // iterations of a phase before a stall may end it
constexpr int kMaxCheckGap = 48;  // most iterations between two checks
constexpr int kRateSpan = 4;      // iterations the decay rate is measured over, where checks allow

struct CheckSchedule {
  int every = 0;
  int next = 0;
  int last_t = -1;
  double last_rho = -1.0;
  double need = -1.0;  // predicted iterations to `tol` at the last check (-1: no prediction)
  std::vector<std::pair<int, double>> hist;  // (t, rho) of the earlier checks of this phase
  int plan(int t, double rho, double tol) {
    need = -1.0;
    if (every > 0) return next = t + every;
    // decay rate against the latest check at least kRateSpan iterations back
    // where there is one (the maximum over the triplets moves unevenly from
    // one iteration to the next), else against the last check
    int bt = last_t;
    double br = last_rho;
    for (auto it = hist.rbegin(); it != hist.rend(); ++it)
      if (it->first <= t - kRateSpan) {
        bt = it->first;
        br = it->second;
        break;
      }
    int gap = 4;   // after the first check: the early decay is not yet geometric
    if (bt >= 0 && rho > 0.0 && br > rho) {
      const double rate = std::pow(rho / br, 1.0 / (t - bt));
      need = std::log(tol / rho) / std::log(rate);
      gap = static_cast<int>(0.9 * need);
    } else if (last_t >= 0) {
      gap = 2 * (t - last_t);
    }
    gap = gap < 1 ? 1 : (gap > kMaxCheckGap ? kMaxCheckGap : gap);
    hist.emplace_back(t, rho);
    last_t = t;
    last_rho = rho;
    return next = t + gap;
  }
};

// Runs iterations in storage type T from the current Qc.  Returns 1 when the
// Ritz triplets held in st satisfy the stopping rule of this phase (tolerance
// `tol`, or the fixed count), 0 when max_iter was reached.
// stall_rate > 0: also stop (returning 2) when rho has fallen by less than a
// factor stall_rate per iteration since the previous check -- the precision
// floor of the block storage has been reached.  phase_cap > 0: stop (2) after
// that iteration.  probe: stop (3) at the first check that predicts the
// iterations still needed (st.probe_need).
template <typename T>
int run_phase(SvdState& st, isvd_operator* op, const isvd_svd_params* prm, double tol, bool fixed, int t0,
              hipStream_t stream, double stall_rate = 0.0, int phase_cap = 0, bool probe = false) {
  const int l = st.l;
  CheckSchedule sched;
  sched.every = prm->check_every > 0 ? prm->check_every : 0;
  sched.next = t0 + (sched.every > 0 ? 0 : kFirstCheck);
  // 1^T Q of the blocks fed to the NE products come from the orthonormaliser
  const bool ne = op->form == ISVD_FORM_NE;
  if (ne) {
    st.sum_c.ensure(static_cast<size_t>(l) * sizeof(double));
    st.sum_r.ensure(static_cast<size_t>(l) * sizeof(double));
  }
  bool qc_sums = false;  // sum_c holds 1^T Qc (false for the start block)
  for (int t = t0;; ++t) {
    T* Y = st.y.as<T>();
    void* tok = phase_begin(kPhaseProduct, stream);
    apply_operator<T>(op, false, st.qc.as<T>(), st.ld, l, Y, st.ld, stream, qc_sums ? st.sum_c.as<double>() : nullptr);
    phase_end(stream, tok);
    st.applies++;
    if (!fixed && st.have_ritz && st.ritz_iter == t - 1) {
      tok = phase_begin(kPhaseCheck, stream);
      st.residual = residual<T>(st, Y, stream);
      phase_end(stream, tok);
      trace_check(st, std::is_same<T, bf16>::value ? "bf16" : (std::is_same<T, float>::value ? "fp32" : "fp64"), t - 1);
      if (st.residual <= tol) {
        st.iterations = t - 1;
        return 1;
      }
      // precision floor: less than (1 - stall_rate) improvement per iteration
      // since the previous check (checks near the target can be 1-3 iterations
      // apart); not in the first kStallMinIter iterations of the phase, where
      // the worst triplet's residual can stand still while the basis rotates
      if (stall_rate > 0.0 && sched.last_rho > 0.0 && sched.last_t >= 0 && (t - 1) - t0 >= kStallMinIter &&
          st.residual > sched.last_rho * std::pow(stall_rate, static_cast<double>((t - 1) - sched.last_t))) {
        st.iterations = t - 1;
        return 2;
      }
      sched.plan(t - 1, st.residual, tol);
      // probe: stop (returning 3) once the decay rate predicts the rest
      if (probe && sched.need > 0.0) {
        st.iterations = t - 1;
        st.probe_need = static_cast<int>(std::ceil(sched.need));
        return 3;
      }
    }
    if (!fixed && phase_cap > 0 && t >= phase_cap && st.have_ritz && st.ritz_iter == t - 1) {
      st.iterations = t - 1;
      return 2;
    }
    if (!fixed && t >= prm->max_iter) {
      // out of iterations: return the triplets of the last finished iteration
      if (st.ritz_iter != t - 1 && t >= 1) {
        tok = phase_begin(kPhaseRitz, stream);
        ritz(st, stream, kRitzTol<T>);
        phase_end(stream, tok);
        st.ritz_iter = t - 1;
      }
      st.iterations = t - 1;
      return 0;
    }
    // Rayleigh-Ritz at the end of this iteration needs orthonormal Qr, Qc (CholeskyQR2);
    // otherwise one Cholesky pass (Algorithm 2) keeps the span, which is all the next product needs
    const bool ritz_now = fixed ? (t >= prm->q)
                                : (t >= sched.next || (phase_cap > 0 && t + 1 >= phase_cap) || t + 1 >= prm->max_iter);
    const int np_ = ritz_now || prm->orth_passes >= 2 ? 2 : 1;
    tok = phase_begin(kPhaseOrth, stream);
    orthonormalize<T>(st, Y, st.r, nullptr, ne ? st.sum_r.as<double>() : nullptr, stream, np_);
    phase_end(stream, tok);
    std::swap(st.qr.p, st.y.p);
    std::swap(st.qr.bytes, st.y.bytes);
    tok = phase_begin(kPhaseProduct, stream);
    apply_operator<T>(op, true, st.qr.as<T>(), st.ld, l, st.w.as<T>(), st.ld, stream, ne ? st.sum_r.as<double>() : nullptr);
    phase_end(stream, tok);
    st.applies++;
    tok = phase_begin(kPhaseOrth, stream);
    orthonormalize<T>(st, st.w.as<T>(), st.c, st.Rc.as<double>(), ne ? st.sum_c.as<double>() : nullptr, stream, np_);
    phase_end(stream, tok);
    std::swap(st.qc.p, st.w.p);
    std::swap(st.qc.bytes, st.w.bytes);
    qc_sums = ne;
    if ((fixed && t >= prm->q) || (!fixed && ritz_now)) {
      tok = phase_begin(kPhaseRitz, stream);
      ritz(st, stream, kRitzTol<T>);
      phase_end(stream, tok);
      st.ritz_iter = t;
    }
    if (fixed && t >= prm->q) {
      st.iterations = t;
      return 1;
    }
  }
}

// Blocks of st from storage S to storage D: Qc converted, the other blocks
// reallocated; the Ritz state of the old storage is dropped.
template <typename D, typename S>
void switch_storage(SvdState& st, hipStream_t stream) {
  DevBuf qcn;
  qcn.ensure(static_cast<size_t>(st.c) * st.ld * sizeof(D));
  launch_convert<D, S>(st.c, st.l, st.qc.as<S>(), st.ld, qcn.as<D>(), st.ld, stream);
  ISVD_HIP(hipStreamSynchronize(stream));
  st.qc.release();
  st.w.release();
  st.qr.release();
  st.y.release();
  std::swap(st.qc.p, qcn.p);
  std::swap(st.qc.bytes, qcn.bytes);
  st.w.ensure(static_cast<size_t>(st.c) * st.ld * sizeof(D));
  st.qr.ensure(static_cast<size_t>(st.r) * st.ld * sizeof(D));
  st.y.ensure(static_cast<size_t>(st.r) * st.ld * sizeof(D));
  st.have_ritz = false;
  st.ritz_iter = -1;
}

template <typename T>
void load_start_block(SvdState& st, const isvd_svd_params* prm, hipStream_t stream) {
  if (prm->omega) {
    launch_convert<T, T>(st.c, st.l, static_cast<const T*>(prm->omega), prm->ld_omega, st.qc.as<T>(), st.ld, stream);
  } else {
    launch_gaussian<T>(st.c, st.l, prm->seed, st.qc.as<T>(), st.ld, stream);
  }
}

template <typename T>
isvd_status svd_same_precision(isvd_operator* op, const isvd_svd_params* prm, void* U, int64_t ldu, double* S,
                               void* V, int64_t ldv, SvdState& st, hipStream_t stream) {
  ensure_blocks<T>(st);
  load_start_block<T>(st, prm, stream);
  const bool fixed = !(prm->tol > 0.0);
  const int ok = run_phase<T>(st, op, prm, prm->tol, fixed, 0, stream);
  finalize<T, T>(st, op, U, ldu, S, V, ldv, stream);
  return ok ? ISVD_OK : ISVD_E_NOT_CONVERGED;
}

isvd_status svd_bf16(isvd_operator* op, const isvd_svd_params* prm, void* U, int64_t ldu, double* S, void* V,
                     int64_t ldv, SvdState& st, hipStream_t stream) {
  ensure_blocks<bf16>(st);
  load_start_block<bf16>(st, prm, stream);
  const bool fixed = !(prm->tol > 0.0);
  if (fixed || !(prm->fp32_switch_tol > 0.0)) {
    const int ok = run_phase<bf16>(st, op, prm, prm->tol, fixed, 0, stream);
    st.bf16_iterations = st.iterations + 1;
    finalize<bf16, float>(st, op, U, ldu, S, V, ldv, stream);
    return ok ? ISVD_OK : ISVD_E_NOT_CONVERGED;
  }
  // BF16 until rho <= fp32_switch_tol or the residual stalls (or for
  // bf16_max_iter iterations), then FP32.
  const bool auto_len = prm->bf16_max_iter <= 0;
  const int ok16 = run_phase<bf16>(st, op, prm, prm->fp32_switch_tol, false, 0, stream, auto_len ? 0.98 : 0.0,
                                  prm->bf16_max_iter);
  if (!ok16) {
    st.bf16_iterations = st.iterations + 1;
    finalize<bf16, float>(st, op, U, ldu, S, V, ldv, stream);
    return ISVD_E_NOT_CONVERGED;
  }
  // The BF16 phase stopped with Qc of iteration t - 1 and one extra product;
  // the next phase restarts from that Qc.
  int t = st.iterations + 1;
  int bf16_its = t;
  switch_storage<float, bf16>(st, stream);
  // With the automatic switch, the residual seen in BF16 may be the floor of
  // the BF16 rounding of the blocks (amplified by the largest singular value)
  // while the subspace itself still converges as fast as in FP32.  A short
  // FP32 probe measures the true residual and its decay; while the predicted
  // rest exceeds the FP32 iterations needed after a BF16 stretch (kPolish) by
  // at least kMinBack, the blocks go back to BF16 for the difference (at most
  // as many iterations as done so far), then the probe repeats.  The early
  // FP32 decay is a little faster than the later one, so the prediction is
  // taken 10% longer.
  constexpr int kPolish = 10, kMinBack = 8, kMaxRounds = 3;
  constexpr double kNeedMargin = 1.1;
  for (int round = 0; auto_len && round < kMaxRounds; ++round) {
    const int pr = run_phase<float>(st, op, prm, prm->tol, false, t, stream, 0.0, 0, true);
    if (pr != 3) {
      st.bf16_iterations = bf16_its;
      finalize<float, float>(st, op, U, ldu, S, V, ldv, stream);
      return pr == 1 ? ISVD_OK : ISVD_E_NOT_CONVERGED;
    }
    t = st.iterations + 1;
    int back = static_cast<int>(std::ceil(kNeedMargin * st.probe_need)) - kPolish;
    back = std::min(back, std::max(16, t));
    back = std::min(back, prm->max_iter - 1 - t - kPolish);
    if (back < kMinBack) break;
    switch_storage<bf16, float>(st, stream);
    isvd_svd_params fixed_prm = *prm;
    fixed_prm.q = t + back - 1;   // iterations t .. t + back - 1, no residual checks
    run_phase<bf16>(st, op, &fixed_prm, 0.0, true, t, stream);
    bf16_its += back;
    t = st.iterations + 1;
    switch_storage<float, bf16>(st, stream);
  }
  st.bf16_iterations = bf16_its;
  const int ok = run_phase<float>(st, op, prm, prm->tol, false, t, stream);
  finalize<float, float>(st, op, U, ldu, S, V, ldv, stream);
  return ok ? ISVD_OK : ISVD_E_NOT_CONVERGED;
}

}  // namespace

isvd_status truncated_svd(isvd_operator* op, const isvd_svd_params* prm, void* U, int64_t ldu, double* S,
                          void* V, int64_t ldv, isvd_svd_info* info, hipStream_t stream) {
  const auto t_start = std::chrono::steady_clock::now();
  ISVD_CHECK(op && prm && U && S && V, ISVD_E_INVALID, "null argument");
  if (!op->svd_cache) op->svd_cache = std::make_shared<SvdState>();
  SvdState& st = *static_cast<SvdState*>(op->svd_cache.get());
  st.reset_counters();
  st.r = op->rows;
  st.c = op->cols;
  st.k = prm->k;
  st.l = prm->k + prm->p;
  const int64_t mn = st.r < st.c ? st.r : st.c;
  ISVD_CHECK(prm->k >= 1 && prm->p >= 0 && st.l <= mn, ISVD_E_INVALID, "need 1 <= k, 0 <= p, k + p <= min(rows, cols)");
  ISVD_CHECK(st.l <= 512, ISVD_E_INVALID, "k + p above 512");
  ISVD_CHECK(prm->q >= 0, ISVD_E_INVALID, "q must be >= 0");
  ISVD_CHECK(!(prm->tol > 0.0) || prm->max_iter >= 1, ISVD_E_INVALID, "tolerance mode needs max_iter >= 1");
  ISVD_CHECK(ldu >= st.k && ldv >= st.k, ISVD_E_INVALID, "ldu/ldv smaller than k");
  ISVD_CHECK(!prm->omega || prm->ld_omega >= st.l, ISVD_E_INVALID, "ld_omega smaller than k + p");
  ISVD_CHECK(prm->orth_method == 0 || prm->orth_method == 1, ISVD_E_INVALID, "orth_method must be 0 or 1");
  st.householder = prm->orth_method == 1;
  st.lp = pad16(st.l);
  st.ld = round_up(st.l, 8);
  clear_chol_flags(st, stream);
  isvd_status rc;
  switch (op->prec) {
    case ISVD_FP64: rc = svd_same_precision<double>(op, prm, U, ldu, S, V, ldv, st, stream); break;
    case ISVD_FP32: rc = svd_same_precision<float>(op, prm, U, ldu, S, V, ldv, st, stream); break;
    default: rc = svd_bf16(op, prm, U, ldu, S, V, ldv, st, stream); break;
  }
  read_chol_flags(st, stream);   // repairs of single passes since the last read
  if (info) {
    info->iterations = st.iterations;
    info->applies = st.applies;
    info->bf16_iterations = op->prec == ISVD_BF16 ? st.bf16_iterations : 0;
    info->residual_checks = st.checks;
    info->used_fallback = st.fallback;
    info->residual = st.residual;
    info->ritz_steps = st.ritz_steps;
    info->jacobi_sweeps = 0;
    if (st.sweeps.p) ISVD_HIP(hipMemcpy(&info->jacobi_sweeps, st.sweeps.p, sizeof(int), hipMemcpyDeviceToHost));
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  }
  if (rc == ISVD_E_NOT_CONVERGED) set_last_error("tolerance not reached within max_iter iterations");
  return rc;
}

// Standalone CholeskyQR2 (or Householder QR) of one block.
template <typename T>
void orthonormalize_block(int64_t rows, int cols, T* Y, int64_t ld, double* Rout, hipStream_t stream,
                          bool householder) {
  SvdState st;
  st.householder = householder;
  st.l = cols;
  st.lp = pad16(cols);
  st.ld = ld;
  st.Rc.ensure(static_cast<size_t>(st.lp) * st.lp * sizeof(double));
  clear_chol_flags(st, stream);
  orthonormalize<T>(st, Y, rows, st.Rc.as<double>(), nullptr, stream);
  if (Rout) {
    launch_convert<double, double>(cols, cols, st.Rc.as<double>(), st.lp, Rout, cols, stream);
  }
  ISVD_HIP(hipStreamSynchronize(stream));
}
template void orthonormalize_block<double>(int64_t, int, double*, int64_t, double*, hipStream_t, bool);
template void orthonormalize_block<float>(int64_t, int, float*, int64_t, double*, hipStream_t, bool);
template void orthonormalize_block<bf16>(int64_t, int, bf16*, int64_t, double*, hipStream_t, bool);

}  // namespace isvd
