// Closed-form learners on a rank-k SVD (Section 3): node embeddings and pair
// scores (Eq. 5), and the least-norm linear model W* = V S^+ U^T Y (Eq. 7),
// multiplied right to left.  Index arrays are checked on the device: an index
// out of range writes NaN where it was used and raises a flag the entry point
// turns into ISVD_E_INVALID (no access outside the arrays).
#include <algorithm>

#include "dense.h"
#include "learners.h"

namespace isvd {

namespace {

unsigned grid_of(int64_t threads) {
  const int64_t g = ceil_div(threads, 256);
  ISVD_CHECK(g <= 0x7fffffff, ISVD_E_INVALID, "learner input too large for one launch");
  return static_cast<unsigned>(g);
}

// out[i][t] = in[i][t] * sqrt(s_t)
template <typename T>
__global__ void embed_kernel(int64_t rows, int k, const T* in, int64_t ldi, const double* s, T* out, int64_t ldo) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= rows * k) return;
  const int64_t i = idx / k;
  const int t = static_cast<int>(idx - i * k);
  out[i * ldo + t] = static_cast<T>(static_cast<double>(in[i * ldi + t]) * sqrt(s[t]));
}

// One 16-lane row per pair: score_p = sum_t U[i_p][t] s_t V[j_p][t], FP64
// products and sums (DPP reduction over the row).  VEC: four FP32 elements
// per lane and step (k and both leading dimensions multiples of 4, 16-byte
// aligned rows).
template <typename T, bool VEC>
__global__ __launch_bounds__(256) void pair_score_kernel(int k, const T* U, int64_t ldu, int64_t nu, const double* s,
                                                          const T* V, int64_t ldv, int64_t nv, int64_t npairs,
                                                          const int64_t* pi, const int64_t* pj, double* scores,
                                                          int* bad) {
  const int64_t p = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 4;
  const int g = threadIdx.x & 15;
  const bool live = p < npairs;
  const int64_t i = live ? pi[p] : 0, j = live ? pj[p] : 0;
  const bool ok = live && i >= 0 && i < nu && j >= 0 && j < nv;
  double acc = 0.0;
  if (ok) {
    const T* ur = U + i * ldu;
    const T* vr = V + j * ldv;
    if constexpr (VEC) {
      for (int t = 4 * g; t < k; t += 64) {
        const float4 a = *reinterpret_cast<const float4*>(ur + t);
        const float4 b = *reinterpret_cast<const float4*>(vr + t);
        acc += static_cast<double>(a.x) * s[t] * static_cast<double>(b.x);
        acc += static_cast<double>(a.y) * s[t + 1] * static_cast<double>(b.y);
        acc += static_cast<double>(a.z) * s[t + 2] * static_cast<double>(b.z);
        acc += static_cast<double>(a.w) * s[t + 3] * static_cast<double>(b.w);
      }
    } else {
      for (int t = g; t < k; t += 16) acc += static_cast<double>(ur[t]) * s[t] * static_cast<double>(vr[t]);
    }
  }
  acc = row16_sum(acc);  // every lane of the wave takes part
  if (live && g == 0) {
    scores[p] = ok ? acc : __builtin_nan("");
    if (!ok) atomicOr(bad, 1);
  }
}

// dst[r][c] = src[rows[r]][c] for c < cols (rows checked; zeros and the flag
// for an index out of range)
template <typename T>
__global__ void gather_rows_kernel(int64_t nsub, int64_t cols, const int64_t* rows, int64_t nsrc, const T* src,
                                   int64_t lds, T* dst, int64_t ldd, int* bad) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= nsub * cols) return;
  const int64_t r = idx / cols, c = idx - r * cols;
  const int64_t sr = rows[r];
  const bool ok = sr >= 0 && sr < nsrc;
  dst[r * ldd + c] = ok ? src[sr * lds + c] : T(0);
  if (!ok && c == 0) atomicOr(bad, 1);
}

// W[j][y] = sum_t V[j][t] s^+_t T[t][y] (FP64), s^+_t = 1/s_t for s_t > rcond
// max(s), else 0.  One wave per row of V, lanes over the label columns.
template <typename T>
__global__ __launch_bounds__(256) void nc_apply_kernel(int64_t rows, int k, int ny, const T* V, int64_t ldv,
                                                        const double* s, double rcond, const double* Tm,
                                                        int64_t ldt, double* W, int64_t ldw) {
  __shared__ double sp[1024];
  __shared__ double smax;
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int t = 0; t < k; ++t) m = fmax(m, s[t]);
    smax = m;
  }
  __syncthreads();
  const double cut = rcond * smax;
  for (int t = threadIdx.x; t < k; t += blockDim.x) sp[t] = s[t] > cut ? 1.0 / s[t] : 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t j = static_cast<int64_t>(blockIdx.x) * 4 + wave; j < rows; j += static_cast<int64_t>(gridDim.x) * 4) {
    const T* vr = V + j * ldv;
    for (int y0 = 0; y0 < ny; y0 += 64) {
      const int y = y0 + lane;
      double acc = 0.0;
      if (y < ny)
        for (int t = 0; t < k; ++t) acc += static_cast<double>(vr[t]) * sp[t] * Tm[static_cast<int64_t>(t) * ldt + y];
      if (y < ny) W[j * ldw + y] = acc;
    }
  }
}

}  // namespace

template <typename T>
void launch_ne_embed(int64_t rows, int k, const T* in, int64_t ldi, const double* s, T* out, int64_t ldo,
                     hipStream_t stream) {
  const int64_t total = rows * k;
  if (total == 0) return;
  hipLaunchKernelGGL(embed_kernel<T>, dim3(grid_of(total)), dim3(256), 0, stream, rows,
                     k, in, ldi, s, out, ldo);
  ISVD_LAUNCH_CHECK();
}
template void launch_ne_embed<float>(int64_t, int, const float*, int64_t, const double*, float*, int64_t, hipStream_t);
template void launch_ne_embed<double>(int64_t, int, const double*, int64_t, const double*, double*, int64_t,
                                      hipStream_t);

template <typename T>
void launch_pair_scores(int k, const T* U, int64_t ldu, int64_t nu, const double* s, const T* V, int64_t ldv,
                        int64_t nv, int64_t npairs, const int64_t* pi, const int64_t* pj, double* scores, int* bad,
                        hipStream_t stream) {
  if (npairs == 0) return;
  const dim3 grid(grid_of(npairs * 16)), block(256);
  bool vec = false;
  if constexpr (std::is_same<T, float>::value)
    vec = k % 4 == 0 && ldu % 4 == 0 && ldv % 4 == 0 && reinterpret_cast<uintptr_t>(U) % 16 == 0 &&
          reinterpret_cast<uintptr_t>(V) % 16 == 0;
  if (vec)
    hipLaunchKernelGGL((pair_score_kernel<T, true>), grid, block, 0, stream, k, U, ldu, nu, s, V, ldv, nv, npairs, pi,
                       pj, scores, bad);
  else
    hipLaunchKernelGGL((pair_score_kernel<T, false>), grid, block, 0, stream, k, U, ldu, nu, s, V, ldv, nv, npairs,
                       pi, pj, scores, bad);
  ISVD_LAUNCH_CHECK();
}
template void launch_pair_scores<float>(int, const float*, int64_t, int64_t, const double*, const float*, int64_t,
                                        int64_t, int64_t, const int64_t*, const int64_t*, double*, int*, hipStream_t);
template void launch_pair_scores<double>(int, const double*, int64_t, int64_t, const double*, const double*, int64_t,
                                         int64_t, int64_t, const int64_t*, const int64_t*, double*, int*,
                                         hipStream_t);

template <typename T>
void launch_gather_rows(int64_t nsub, int64_t cols, const int64_t* rows, int64_t nsrc, const T* src, int64_t lds,
                        T* dst, int64_t ldd, int* bad, hipStream_t stream) {
  const int64_t total = nsub * cols;
  if (total == 0) return;
  hipLaunchKernelGGL(gather_rows_kernel<T>, dim3(grid_of(total)), dim3(256), 0, stream,
                     nsub, cols, rows, nsrc, src, lds, dst, ldd, bad);
  ISVD_LAUNCH_CHECK();
}
template void launch_gather_rows<float>(int64_t, int64_t, const int64_t*, int64_t, const float*, int64_t, float*,
                                        int64_t, int*, hipStream_t);
template void launch_gather_rows<double>(int64_t, int64_t, const int64_t*, int64_t, const double*, int64_t, double*,
                                         int64_t, int*, hipStream_t);

template <typename T>
void launch_nc_apply(int64_t rows, int k, int ny, const T* V, int64_t ldv, const double* s, double rcond,
                     const double* Tm, int64_t ldt, double* W, int64_t ldw, hipStream_t stream) {
  ISVD_CHECK(k >= 1 && k <= 1024, ISVD_E_INVALID, "nc fit: k out of range");
  if (rows == 0 || ny == 0) return;
  const int64_t blocks = std::min<int64_t>(ceil_div(rows, 4), 4096);
  hipLaunchKernelGGL(nc_apply_kernel<T>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, rows, k, ny, V,
                     ldv, s, rcond, Tm, ldt, W, ldw);
  ISVD_LAUNCH_CHECK();
}
template void launch_nc_apply<float>(int64_t, int, int, const float*, int64_t, const double*, double, const double*,
                                     int64_t, double*, int64_t, hipStream_t);
template void launch_nc_apply<double>(int64_t, int, int, const double*, int64_t, const double*, double,
                                      const double*, int64_t, double*, int64_t, hipStream_t);

}  // namespace isvd
