// Householder QR of a tall block (Algorithm 2's first orthonormaliser; the
// baseline the Cholesky pass is compared with in Fig. 3).  Column j:
//   d_k = sum_{i>=j} a_ij a_ik  (k >= j; FP64 sums, one pass over the trailing rows)
//   alpha = -sign(a_jj) sqrt(d_j), v = a_j - alpha e_j, beta = 2 / v^T v,
//   g_k = beta (d_k - alpha a_jk)   (= beta v^T a_k, k > j)
//   a_ik -= v_i g_k                 (i >= j, k > j; row j becomes row j of R)
// with v kept in column j (a_jj <- v_j).  Q = H_0 ... H_{l-1} [I; 0] is then
// formed backwards in a separate block: z_k = v^T q_k, q_k -= beta v z_k.
// Unblocked (two passes over the trailing block per column and per
// reflector): a reference point for the cost of an orthonormalisation, not
// the iteration's default.
#include <algorithm>

#include "householder.h"

namespace isvd {

namespace {

constexpr int kHhThreads = 256;
constexpr int kHhMaxCols = 1024;
constexpr int kHhPer = kHhMaxCols / 64;   // columns per lane at most
constexpr int kHhMaxParts = 1024;          // row slices of the dot-product pass

// partial[b][k] = sum over this block's rows i >= j of V[i][j] W[i][k], k in [col0, l)
template <typename T>
__global__ __launch_bounds__(kHhThreads) void hh_dots_kernel(int64_t rows, int l, int j, int col0, const T* V,
                                                             int64_t ldv, const T* W, int64_t ldw,
                                                             int64_t rows_per_block, double* partial) {
  __shared__ double red[kHhThreads / 64][kHhMaxCols];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = j + static_cast<int64_t>(blockIdx.x) * rows_per_block;
  const int64_t r1 = std::min<int64_t>(r0 + rows_per_block, rows);
  double acc[kHhPer];
#pragma unroll
  for (int c = 0; c < kHhPer; ++c) acc[c] = 0.0;
  // four rows per step: their loads are independent and in flight together
  constexpr int kRows = 4;
  for (int64_t i0 = r0 + wave * kRows; i0 < r1; i0 += (kHhThreads / 64) * kRows) {
    double vi[kRows];
    const T* w[kRows];
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
      const int64_t i = i0 + q < r1 ? i0 + q : r0;
      vi[q] = i0 + q < r1 ? static_cast<double>(Elem<T>::load(V + i * ldv + j)) : 0.0;
      w[q] = W + i * ldw;
    }
#pragma unroll
    for (int c = 0; c < kHhPer; ++c) {
      const int k = col0 + lane + 64 * c;
      if (k < l) {
#pragma unroll
        for (int q = 0; q < kRows; ++q) acc[c] += vi[q] * static_cast<double>(Elem<T>::load(w[q] + k));
      }
    }
  }
#pragma unroll
  for (int c = 0; c < kHhPer; ++c) {
    const int k = col0 + lane + 64 * c;
    if (k < l) red[wave][k] = acc[c];
  }
  __syncthreads();
  for (int k = col0 + static_cast<int>(threadIdx.x); k < l; k += kHhThreads) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kHhThreads / 64; ++w) s += red[w][k];
    partial[static_cast<int64_t>(blockIdx.x) * l + k] = s;
  }
}

// sum over p < nparts of partial[p][k], four sums with several loads in flight
__device__ inline double sum_parts(const double* partial, int nparts, int l, int k) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int p = 0;
#pragma unroll 2
  for (; p + 3 < nparts; p += 4) {
    s0 += partial[static_cast<int64_t>(p) * l + k];
    s1 += partial[static_cast<int64_t>(p + 1) * l + k];
    s2 += partial[static_cast<int64_t>(p + 2) * l + k];
    s3 += partial[static_cast<int64_t>(p + 3) * l + k];
  }
  for (; p < nparts; ++p) s0 += partial[static_cast<int64_t>(p) * l + k];
  return (s0 + s1) + (s2 + s3);
}

// Reflector of column j from the reduced dot products (one block).
template <typename T>
__global__ __launch_bounds__(kHhThreads) void hh_reflect_kernel(int l, int j, int nparts, const double* partial,
                                                                T* Y, int64_t ld, double* g, double* alpha,
                                                                double* beta) {
  __shared__ double d[kHhMaxCols];
  __shared__ double sh[2];
  for (int k = j + static_cast<int>(threadIdx.x); k < l; k += kHhThreads) d[k] = sum_parts(partial, nparts, l, k);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double ajj = static_cast<double>(Elem<T>::load(Y + static_cast<int64_t>(j) * ld + j));
    const double nrm = sqrt(d[j]);
    const double a = ajj >= 0.0 ? -nrm : nrm;
    const double vtv = 2.0 * (d[j] - a * ajj);
    const double b = vtv > 0.0 ? 2.0 / vtv : 0.0;
    sh[0] = a;
    sh[1] = b;
    alpha[j] = a;
    beta[j] = b;
    Elem<T>::store(Y + static_cast<int64_t>(j) * ld + j, static_cast<typename ComputeOf<T>::type>(ajj - a));  // v_j
  }
  __syncthreads();
  const double a = sh[0], b = sh[1];
  for (int k = j + 1 + static_cast<int>(threadIdx.x); k < l; k += kHhThreads)
    g[k] = b * (d[k] - a * static_cast<double>(Elem<T>::load(Y + static_cast<int64_t>(j) * ld + k)));
}

// g_k = beta_j z_k for the backward formation of Q (one block).
__global__ __launch_bounds__(kHhThreads) void hh_scale_kernel(int l, int j, int nparts, const double* partial,
                                                              const double* beta, double* g) {
  for (int k = j + static_cast<int>(threadIdx.x); k < l; k += kHhThreads) g[k] = beta[j] * sum_parts(partial, nparts, l, k);
}

// W[i][k] -= V[i][j] g_k for rows i >= j, columns k in [col0, l): one wave per row.
template <typename T>
__global__ __launch_bounds__(kHhThreads) void hh_update_kernel(int64_t rows, int l, int j, int col0, const T* V,
                                                               int64_t ldv, T* W, int64_t ldw, const double* g) {
  using C = typename ComputeOf<T>::type;
  const int lane = threadIdx.x & 63;
  for (int64_t i = j + ((static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6); i < rows;
       i += (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6) {
    const C vi = static_cast<C>(Elem<T>::load(V + i * ldv + j));
    T* w = W + i * ldw;
    for (int k = col0 + lane; k < l; k += 64)
      Elem<T>::store(w + k, static_cast<C>(Elem<T>::load(w + k)) - vi * static_cast<C>(g[k]));
  }
}

// Q = [I_l; 0]
template <typename T>
__global__ void hh_eye_kernel(int64_t rows, int l, T* Q, int64_t ldq) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= rows * l) return;
  const int64_t i = idx / l;
  const int k = static_cast<int>(idx - i * l);
  Elem<T>::store(Q + i * ldq + k, static_cast<typename ComputeOf<T>::type>(i == k ? 1.0 : 0.0));
}

// R (lp x lp, FP64): alpha on the diagonal, the reduced rows above it, zeros
// below, identity on the padding diagonal.
template <typename T>
__global__ void hh_extract_r_kernel(int l, int lp, const T* Y, int64_t ld, const double* alpha, double* R) {
  const int idx = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  if (idx >= lp * lp) return;
  const int i = idx / lp, k = idx - (idx / lp) * lp;
  double v = 0.0;
  if (i < l && k < l) {
    if (k == i) v = alpha[i];
    else if (k > i) v = static_cast<double>(Elem<T>::load(Y + static_cast<int64_t>(i) * ld + k));
  } else if (i == k) {
    v = 1.0;
  }
  R[idx] = v;
}

int parts_for(int64_t rows, int j) {
  return static_cast<int>(std::min<int64_t>(kHhMaxParts, std::max<int64_t>(1, ceil_div(rows - j, 64))));
}

}  // namespace

size_t householder_workspace_doubles(int l) {
  return static_cast<size_t>(kHhMaxParts) * l + 3 * static_cast<size_t>(l);
}

template <typename T>
void launch_householder_qr(int64_t rows, int l, T* Y, int64_t ld, T* Q, int64_t ldq, double* R, int lp,
                           double* work, hipStream_t stream) {
  ISVD_CHECK(l >= 1 && l <= kHhMaxCols && rows >= l, ISVD_E_INVALID, "householder: need 1 <= l <= min(rows, 1024)");
  double* partial = work;
  double* g = work + static_cast<size_t>(kHhMaxParts) * l;
  double* alpha = g + l;
  double* beta = alpha + l;
  const unsigned upd_blocks = static_cast<unsigned>(std::min<int64_t>(ceil_div(rows, 4), 16384));
  for (int j = 0; j < l; ++j) {
    const int P = parts_for(rows, j);
    const int64_t rpb = ceil_div(rows - j, P);
    hipLaunchKernelGGL(hh_dots_kernel<T>, dim3(P), dim3(kHhThreads), 0, stream, rows, l, j, j, Y, ld, Y, ld, rpb,
                       partial);
    hipLaunchKernelGGL(hh_reflect_kernel<T>, dim3(1), dim3(kHhThreads), 0, stream, l, j, P, partial, Y, ld, g, alpha,
                       beta);
    if (j + 1 < l)
      hipLaunchKernelGGL(hh_update_kernel<T>, dim3(upd_blocks), dim3(kHhThreads), 0, stream, rows, l, j, j + 1, Y, ld,
                         Y, ld, g);
  }
  ISVD_LAUNCH_CHECK();
  if (R)
    hipLaunchKernelGGL(hh_extract_r_kernel<T>, dim3(static_cast<unsigned>(ceil_div(static_cast<int64_t>(lp) * lp, 256))),
                       dim3(256), 0, stream, l, lp, Y, ld, alpha, R);
  hipLaunchKernelGGL(hh_eye_kernel<T>, dim3(static_cast<unsigned>(ceil_div(rows * l, 256))), dim3(256), 0, stream,
                     rows, l, Q, ldq);
  for (int j = l - 1; j >= 0; --j) {
    const int P = parts_for(rows, j);
    const int64_t rpb = ceil_div(rows - j, P);
    hipLaunchKernelGGL(hh_dots_kernel<T>, dim3(P), dim3(kHhThreads), 0, stream, rows, l, j, j, Y, ld, Q, ldq, rpb,
                       partial);
    hipLaunchKernelGGL(hh_scale_kernel, dim3(1), dim3(kHhThreads), 0, stream, l, j, P, partial, beta, g);
    hipLaunchKernelGGL(hh_update_kernel<T>, dim3(upd_blocks), dim3(kHhThreads), 0, stream, rows, l, j, j, Y, ld, Q,
                       ldq, g);
  }
  ISVD_LAUNCH_CHECK();
}
template void launch_householder_qr<double>(int64_t, int, double*, int64_t, double*, int64_t, double*, int, double*,
                                            hipStream_t);
template void launch_householder_qr<float>(int64_t, int, float*, int64_t, float*, int64_t, double*, int, double*,
                                           hipStream_t);
template void launch_householder_qr<bf16>(int64_t, int, bf16*, int64_t, bf16*, int64_t, double*, int, double*,
                                          hipStream_t);

}  // namespace isvd
