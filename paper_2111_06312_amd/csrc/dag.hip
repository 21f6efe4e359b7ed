// Block kernels of the symbolic-matrix evaluator: Y = alpha X + beta Y and
// Y = diag(d) X.  One wave per row, lanes over the columns.
#include <algorithm>

#include "dag.h"

namespace isvd {

namespace {

unsigned row_blocks(int64_t rows) { return static_cast<unsigned>(std::min<int64_t>(ceil_div(rows, 4), 16384)); }

// beta == 0: Y is written without being read
template <typename T>
__global__ __launch_bounds__(256) void axpby_kernel(int64_t rows, int cols, double alpha, const T* X, int64_t ldx,
                                                    double beta, T* Y, int64_t ldy) {
  using C = typename ComputeOf<T>::type;
  const int lane = threadIdx.x & 63;
  const C a = static_cast<C>(alpha), b = static_cast<C>(beta);
  for (int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; i < rows;
       i += (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6) {
    const T* x = X + i * ldx;
    T* y = Y + i * ldy;
    if (beta == 0.0) {
      for (int c = lane; c < cols; c += 64) y[c] = static_cast<T>(a * x[c]);
    } else {
      for (int c = lane; c < cols; c += 64) y[c] = static_cast<T>(a * x[c] + b * y[c]);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void diag_scale_kernel(int64_t rows, int cols, const double* d, const T* X,
                                                         int64_t ldx, T* Y, int64_t ldy) {
  using C = typename ComputeOf<T>::type;
  const int lane = threadIdx.x & 63;
  for (int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; i < rows;
       i += (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6) {
    const C di = static_cast<C>(d[i]);
    const T* x = X + i * ldx;
    T* y = Y + i * ldy;
    for (int c = lane; c < cols; c += 64) y[c] = static_cast<T>(di * x[c]);
  }
}

}  // namespace

template <typename T>
void launch_axpby(int64_t rows, int cols, double alpha, const T* X, int64_t ldx, double beta, T* Y, int64_t ldy,
                  hipStream_t stream) {
  if (rows == 0 || cols == 0) return;
  hipLaunchKernelGGL(axpby_kernel<T>, dim3(row_blocks(rows)), dim3(256), 0, stream, rows, cols, alpha, X, ldx, beta,
                     Y, ldy);
  ISVD_LAUNCH_CHECK();
}
template void launch_axpby<float>(int64_t, int, double, const float*, int64_t, double, float*, int64_t, hipStream_t);
template void launch_axpby<double>(int64_t, int, double, const double*, int64_t, double, double*, int64_t, hipStream_t);

template <typename T>
void launch_diag_scale(int64_t rows, int cols, const double* d, const T* X, int64_t ldx, T* Y, int64_t ldy,
                       hipStream_t stream) {
  if (rows == 0 || cols == 0) return;
  hipLaunchKernelGGL(diag_scale_kernel<T>, dim3(row_blocks(rows)), dim3(256), 0, stream, rows, cols, d, X, ldx, Y,
                     ldy);
  ISVD_LAUNCH_CHECK();
}
template void launch_diag_scale<float>(int64_t, int, const double*, const float*, int64_t, float*, int64_t, hipStream_t);
template void launch_diag_scale<double>(int64_t, int, const double*, const double*, int64_t, double*, int64_t,
                                        hipStream_t);

}  // namespace isvd
