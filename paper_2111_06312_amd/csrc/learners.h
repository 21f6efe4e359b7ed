// Closed-form learners on a rank-k SVD (Section 3): kernels behind the
// isvd_ne_* and isvd_nc_fit entry points.
#pragma once

#include "common.h"

namespace isvd {

// out0 = in0 diag(sqrt(s)) (rows0 x k) and out1 = in1 diag(sqrt(s)) (rows1 x
// k), one launch
template <typename T>
void launch_ne_embed(int k, const double* s, int64_t rows0, const T* in0, int64_t ldi0, T* out0, int64_t ldo0,
                     int64_t rows1, const T* in1, int64_t ldi1, T* out1, int64_t ldo1, hipStream_t stream);

// scores[p] = sum_t U[pi[p]][t] s_t V[pj[p]][t] in FP64; indices outside
// [0, nu) / [0, nv) give NaN and set *bad
template <typename T>
void launch_pair_scores(int k, const T* U, int64_t ldu, int64_t nu, const double* s, const T* V, int64_t ldv,
                        int64_t nv, int64_t npairs, const int64_t* pi, const int64_t* pj, double* scores, int* bad,
                        hipStream_t stream);

// dst0 (nsub x cols0) and dst1 (nsub x cols1) = rows `rows` of src0 and
// src1 (nsrc >= 1 rows each); indices out of range give zero rows and set
// *bad
template <typename T>
void launch_gather_rows(int64_t nsub, const int64_t* rows, int64_t nsrc, int cols0, const T* src0, int64_t lds0,
                        T* dst0, int64_t ldd0, int cols1, const T* src1, int64_t lds1, T* dst1, int64_t ldd1, int* bad,
                        hipStream_t stream);

// W (rows x ny, FP64) = V diag(s^+) Tm, s^+_t = 1/s_t for s_t > rcond max(s), else 0
template <typename T>
void launch_nc_apply(int64_t rows, int k, int ny, const T* V, int64_t ldv, const double* s, double rcond,
                     const double* Tm, int64_t ldt, double* W, int64_t ldw, hipStream_t stream);

}  // namespace isvd
