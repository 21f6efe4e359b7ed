// One fused sparse pass over a tall-skinny block:
//
//   acc_i   = sum_{e in row i} v_e * g_{col(e)} * Src[col(e), :]
//   out_i   = (a0 + a1 r_i) acc_i + (b0 + b1 r_i) Add_i + e * s
//   out2_i  = (c0 + c1 r_i) acc_i                      (optional second output)
//
// v_e = CSR value (1 when absent), g_j = cs_a * colscale_j + cs_b (1 when no
// colscale), r_i = rowscale_i (0 when absent), s = an FP64 row vector of
// length ncols (absent -> 0).  Every Horner step of the design-matrix
// products is one such pass (see operator.cpp).
#pragma once

#include "common.h"

namespace isvd {

struct SpmmPass {
  int64_t n_rows = 0;
  int64_t nnz = 0;  // stored entries (only used for byte accounting)
  const int64_t* indptr = nullptr;
  const int32_t* indices = nullptr;
  const float* values = nullptr;

  const void* src = nullptr;
  int64_t ld_src = 0;
  const void* colscale = nullptr;  // compute type, per node
  double cs_a = 1.0, cs_b = 0.0;

  const void* add = nullptr;
  int64_t ld_add = 0;
  const void* rowscale = nullptr;  // compute type, per row
  double a0 = 1.0, a1 = 0.0, b0 = 0.0, b1 = 0.0, e = 0.0;
  const double* svec = nullptr;

  void* out = nullptr;
  int64_t ld_out = 0;
  void* out2 = nullptr;
  int64_t ld_out2 = 0;
  double c0 = 0.0, c1 = 0.0;

  int ncols = 0;
  // rows longer than heavy_threshold are handled by whole workgroups
  int64_t heavy_threshold = 0;
  const int32_t* heavy_rows = nullptr;
  int64_t n_heavy = 0;
};

// Opt-in event timing of passes (profile.cpp).
bool spmm_profiling();
void* spmm_profile_begin(hipStream_t stream, double gather_bytes, double compulsory_bytes, int elem_bytes);
void spmm_profile_end(hipStream_t stream, void* token);
void spmm_profile_enable(bool on);
// elem_bytes != 0: only the passes over blocks of that element size; clear:
// drop the records afterwards.
void spmm_profile_read(double* ms, double* gather, double* compulsory, int64_t* launches, int elem_bytes = 0,
                       bool clear = true);

// Timed regions of other kernels (classes 1 .. kProfileClasses - 1), recorded
// while spmm_profiling() is on: classes 1..3 the learner calls, classes
// kPhaseFirst.. the phases of a truncated SVD (the products with M and M^T,
// orthonormalisation, Rayleigh-Ritz, residual checks, the output products).
constexpr int kLearnerClasses = 3;
constexpr int kPhaseFirst = 1 + kLearnerClasses;
enum Phase { kPhaseProduct = kPhaseFirst, kPhaseOrth, kPhaseRitz, kPhaseCheck, kPhaseOutput };
constexpr int kPhaseCount = 5;
constexpr int kProfileClasses = kPhaseFirst + kPhaseCount;
void* profile_begin(int cls, hipStream_t stream, double bytes, double bytes2, int tag = 0);
void profile_end(hipStream_t stream, void* token);
void profile_read(int cls, double* ms, double* bytes, double* bytes2, int64_t* launches, int tag = 0,
                  bool clear = true);

// Launch one pass; T = storage type (double, float, bf16).
template <typename T>
void launch_spmm_pass(const SpmmPass& p, hipStream_t stream);

// Per-column FP64 sums s = 1^T Y of a rows x cols block (deterministic
// two-stage reduction; partial has room for kColsumBlocks * cols doubles).
constexpr int kColsumBlocks = 1024;
template <typename T>
void launch_colsum(int64_t rows, int cols, const T* y, int64_t ld, double* partial, double* s,
                   hipStream_t stream);

}  // namespace isvd
