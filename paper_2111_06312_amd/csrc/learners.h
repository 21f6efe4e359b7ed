// Closed-form learners on a rank-k SVD (Section 3): kernels behind the
// isvd_ne_* and isvd_nc_fit entry points.
#pragma once

#include "common.h"

namespace isvd {

// out = in diag(sqrt(s)) (rows x k)
template <typename T>
void launch_ne_embed(int64_t rows, int k, const T* in, int64_t ldi, const double* s, T* out, int64_t ldo,
                     hipStream_t stream);

// scores[p] = sum_t U[pi[p]][t] s_t V[pj[p]][t] in FP64; indices outside
// [0, nu) / [0, nv) give NaN and set *bad
template <typename T>
void launch_pair_scores(int k, const T* U, int64_t ldu, int64_t nu, const double* s, const T* V, int64_t ldv,
                        int64_t nv, int64_t npairs, const int64_t* pi, const int64_t* pj, double* scores, int* bad,
                        hipStream_t stream);

// dst (nsub x cols) = rows `rows` of src (nsrc rows); indices out of range
// give zero rows and set *bad
template <typename T>
void launch_gather_rows(int64_t nsub, int64_t cols, const int64_t* rows, int64_t nsrc, const T* src, int64_t lds,
                        T* dst, int64_t ldd, int* bad, hipStream_t stream);

// W (rows x ny, FP64) = V diag(s^+) Tm, s^+_t = 1/s_t for s_t > rcond max(s), else 0
template <typename T>
void launch_nc_apply(int64_t rows, int k, int ny, const T* V, int64_t ldv, const double* s, double rcond,
                     const double* Tm, int64_t ldt, double* W, int64_t ldw, hipStream_t stream);

}  // namespace isvd
