// Graph ingest kernels: self-loop CSR, degrees, D^-1 and (D+I)^-1/2 scales,
// hub-row lists, and the small rearrangements of the feature form.
#include <algorithm>

#include "operator.h"

namespace isvd {

namespace {

__global__ void loops_indptr_kernel(int64_t n, const int64_t* indptr, int64_t* out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i > n) return;
  out[i] = indptr[i] + i;
}

// Row i of A + I: the entries of A with (i, 1) inserted in column order.
__global__ void loops_fill_kernel(int64_t n, const int64_t* indptr, const int32_t* indices,
                                  const float* values, const int64_t* out_ptr, int32_t* out_idx,
                                  float* out_val) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = indptr[i], e = indptr[i + 1];
  int64_t o = out_ptr[i];
  bool placed = false;
  for (int64_t k = b; k < e; ++k) {
    const int32_t c = indices[k];
    if (!placed && c > i) {
      out_idx[o] = static_cast<int32_t>(i);
      if (out_val) out_val[o] = 1.0f;
      ++o;
      placed = true;
    }
    out_idx[o] = c;
    if (out_val) out_val[o] = values ? values[k] : 1.0f;
    ++o;
  }
  if (!placed) {
    out_idx[o] = static_cast<int32_t>(i);
    if (out_val) out_val[o] = 1.0f;
  }
}

// d_i = sum of row i (FP64), then scale_i = 1/d_i (0 if d_i == 0) or d_i^-1/2.
template <typename C>
__global__ void row_scale_kernel(int64_t n, const int64_t* indptr, const float* values, int mode,
                                 double* deg, C* scale) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = indptr[i], e = indptr[i + 1];
  double d = 0.0;
  if (values) {
    for (int64_t k = b; k < e; ++k) d += static_cast<double>(values[k]);
  } else {
    d = static_cast<double>(e - b);
  }
  deg[i] = d;
  double s;
  if (mode == 0) s = d != 0.0 ? 1.0 / d : 0.0;
  else s = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  scale[i] = static_cast<C>(s);
}

__global__ void heavy_rows_kernel(int64_t n, const int64_t* indptr, int64_t threshold, int32_t* list,
                                  unsigned long long* count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (indptr[i + 1] - indptr[i] > threshold) {
    const unsigned long long slot = atomicAdd(count, 1ull);
    list[slot] = static_cast<int32_t>(i);
  }
}

// B[a][j*l + c] = G[j*d + a][c]   (stack of blocks -> side by side), compute type.
template <typename T, typename C>
__global__ void stack_to_side_kernel(int d, int L1, int l, const T* G, int64_t ldg, C* B, int64_t ldb) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(d) * L1 * l) return;
  const int a = static_cast<int>(idx / (static_cast<int64_t>(L1) * l));
  const int rem = static_cast<int>(idx % (static_cast<int64_t>(L1) * l));
  const int j = rem / l, c = rem % l;
  B[static_cast<int64_t>(a) * ldb + rem] = static_cast<C>(Elem<T>::load(G + static_cast<int64_t>(j * d + a) * ldg + c));
}

// out[j*d + a][c] = Cm[a][j*l + c]  (FP64 -> storage type)
template <typename T>
__global__ void side_to_stack_kernel(int d, int L1, int l, const double* Cm, int64_t ldc, T* out, int64_t ldo) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(d) * L1 * l) return;
  const int a = static_cast<int>(idx / (static_cast<int64_t>(L1) * l));
  const int rem = static_cast<int>(idx % (static_cast<int64_t>(L1) * l));
  const int j = rem / l, c = rem % l;
  using C = typename ComputeOf<T>::type;
  Elem<T>::store(out + static_cast<int64_t>(j * d + a) * ldo + c, static_cast<C>(Cm[static_cast<int64_t>(a) * ldc + rem]));
}

// Row selection of an implicit row gather: pos[i] = r for i = rows[r], -1
// for rows not selected.  flag |= 1 for an index out of range, 2 for a
// repeated index.
__global__ void fill_pos_kernel(int64_t n, int32_t* pos) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) pos[i] = -1;
}
__global__ void select_rows_kernel(int64_t nsel, const int64_t* rows, int64_t n, int32_t* pos, int* flag) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= nsel) return;
  const int64_t i = rows[r];
  if (i < 0 || i >= n) {
    atomicOr(flag, 1);
    return;
  }
  if (atomicCAS(pos + i, -1, static_cast<int32_t>(r)) != -1) atomicOr(flag, 2);
}

// dst[r] = src[rows[r]] (ncols elements per row): one wave per row.
template <typename T>
__global__ __launch_bounds__(256) void gather_block_kernel(int64_t nsel, int ncols, const int64_t* rows, const T* src,
                                                           int64_t lds, T* dst, int64_t ldd) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; r < nsel;
       r += (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6) {
    const T* a = src + rows[r] * lds;
    T* o = dst + r * ldd;
    for (int c = lane; c < ncols; c += 64) o[c] = a[c];
  }
}

// dst[i] = src[pos[i]] for selected rows, zeros for the others (every one of
// the n rows written once): one wave per row.
template <typename T>
__global__ __launch_bounds__(256) void scatter_block_kernel(int64_t n, int ncols, const int32_t* pos, const T* src,
                                                            int64_t lds, T* dst, int64_t ldd) {
  const int lane = threadIdx.x & 63;
  for (int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; i < n;
       i += (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6) {
    const int32_t p = pos[i];
    T* o = dst + i * ldd;
    if (p >= 0) {
      const T* a = src + static_cast<int64_t>(p) * lds;
      for (int c = lane; c < ncols; c += 64) o[c] = a[c];
    } else {
      for (int c = lane; c < ncols; c += 64) o[c] = T{};
    }
  }
}

unsigned blocks_for(int64_t n, int t = 256) { return static_cast<unsigned>(ceil_div(n > 0 ? n : 1, t)); }

unsigned row_wave_blocks(int64_t rows) { return static_cast<unsigned>(std::min<int64_t>(ceil_div(rows, 4), 16384)); }

}  // namespace

void build_row_selection(int64_t n, int64_t nsel, const int64_t* rows, int32_t* pos, int* flag, hipStream_t stream) {
  hipLaunchKernelGGL(fill_pos_kernel, dim3(blocks_for(n)), dim3(256), 0, stream, n, pos);
  ISVD_LAUNCH_CHECK();
  if (nsel == 0) return;
  hipLaunchKernelGGL(select_rows_kernel, dim3(blocks_for(nsel)), dim3(256), 0, stream, nsel, rows, n, pos, flag);
  ISVD_LAUNCH_CHECK();
}

template <typename T>
void launch_gather_block(int64_t nsel, int ncols, const int64_t* rows, const T* src, int64_t lds, T* dst,
                         int64_t ldd, hipStream_t stream) {
  if (nsel == 0) return;
  hipLaunchKernelGGL(gather_block_kernel<T>, dim3(row_wave_blocks(nsel)), dim3(256), 0, stream, nsel, ncols, rows,
                     src, lds, dst, ldd);
  ISVD_LAUNCH_CHECK();
}
template void launch_gather_block<double>(int64_t, int, const int64_t*, const double*, int64_t, double*, int64_t, hipStream_t);
template void launch_gather_block<float>(int64_t, int, const int64_t*, const float*, int64_t, float*, int64_t, hipStream_t);
template void launch_gather_block<bf16>(int64_t, int, const int64_t*, const bf16*, int64_t, bf16*, int64_t, hipStream_t);

template <typename T>
void launch_scatter_block(int64_t n, int ncols, const int32_t* pos, const T* src, int64_t lds, T* dst, int64_t ldd,
                          hipStream_t stream) {
  hipLaunchKernelGGL(scatter_block_kernel<T>, dim3(row_wave_blocks(n)), dim3(256), 0, stream, n, ncols, pos, src,
                     lds, dst, ldd);
  ISVD_LAUNCH_CHECK();
}
template void launch_scatter_block<double>(int64_t, int, const int32_t*, const double*, int64_t, double*, int64_t, hipStream_t);
template void launch_scatter_block<float>(int64_t, int, const int32_t*, const float*, int64_t, float*, int64_t, hipStream_t);
template void launch_scatter_block<bf16>(int64_t, int, const int32_t*, const bf16*, int64_t, bf16*, int64_t, hipStream_t);

void build_loop_csr(int64_t n, const int64_t* indptr, const int32_t* indices, const float* values,
                    int64_t nnz, DevBuf& out_ptr, DevBuf& out_idx, DevBuf& out_val, hipStream_t stream) {
  out_ptr.ensure((n + 1) * sizeof(int64_t));
  out_idx.ensure((nnz + n) * sizeof(int32_t));
  if (values) out_val.ensure((nnz + n) * sizeof(float));
  hipLaunchKernelGGL(loops_indptr_kernel, dim3(blocks_for(n + 1)), dim3(256), 0, stream, n, indptr,
                     out_ptr.as<int64_t>());
  ISVD_LAUNCH_CHECK();
  hipLaunchKernelGGL(loops_fill_kernel, dim3(blocks_for(n)), dim3(256), 0, stream, n, indptr, indices,
                     values, out_ptr.as<int64_t>(), out_idx.as<int32_t>(),
                     values ? out_val.as<float>() : nullptr);
  ISVD_LAUNCH_CHECK();
}

template <typename C>
void build_row_scale(int64_t n, const int64_t* indptr, const float* values, int mode, double* deg, C* scale,
                     hipStream_t stream) {
  hipLaunchKernelGGL((row_scale_kernel<C>), dim3(blocks_for(n)), dim3(256), 0, stream, n, indptr, values,
                     mode, deg, scale);
  ISVD_LAUNCH_CHECK();
}
template void build_row_scale<float>(int64_t, const int64_t*, const float*, int, double*, float*, hipStream_t);
template void build_row_scale<double>(int64_t, const int64_t*, const float*, int, double*, double*, hipStream_t);

int64_t build_heavy_rows(int64_t n, const int64_t* indptr, int64_t threshold, DevBuf& list, hipStream_t stream) {
  list.ensure((n > 0 ? n : 1) * sizeof(int32_t));
  DevBuf cnt;
  cnt.ensure(sizeof(unsigned long long));
  ISVD_HIP(hipMemsetAsync(cnt.p, 0, sizeof(unsigned long long), stream));
  hipLaunchKernelGGL(heavy_rows_kernel, dim3(blocks_for(n)), dim3(256), 0, stream, n, indptr, threshold,
                     list.as<int32_t>(), cnt.as<unsigned long long>());
  ISVD_LAUNCH_CHECK();
  unsigned long long h = 0;
  ISVD_HIP(hipMemcpyAsync(&h, cnt.p, sizeof(h), hipMemcpyDeviceToHost, stream));
  ISVD_HIP(hipStreamSynchronize(stream));
  return static_cast<int64_t>(h);
}

template <typename T, typename C>
void launch_stack_to_side(int d, int L1, int l, const T* G, int64_t ldg, C* B, int64_t ldb, hipStream_t stream) {
  hipLaunchKernelGGL((stack_to_side_kernel<T, C>), dim3(blocks_for(static_cast<int64_t>(d) * L1 * l)), dim3(256),
                     0, stream, d, L1, l, G, ldg, B, ldb);
  ISVD_LAUNCH_CHECK();
}
template void launch_stack_to_side<double, double>(int, int, int, const double*, int64_t, double*, int64_t, hipStream_t);
template void launch_stack_to_side<float, float>(int, int, int, const float*, int64_t, float*, int64_t, hipStream_t);
template void launch_stack_to_side<bf16, float>(int, int, int, const bf16*, int64_t, float*, int64_t, hipStream_t);

template <typename T>
void launch_side_to_stack(int d, int L1, int l, const double* Cm, int64_t ldc, T* out, int64_t ldo, hipStream_t stream) {
  hipLaunchKernelGGL((side_to_stack_kernel<T>), dim3(blocks_for(static_cast<int64_t>(d) * L1 * l)), dim3(256), 0,
                     stream, d, L1, l, Cm, ldc, out, ldo);
  ISVD_LAUNCH_CHECK();
}
template void launch_side_to_stack<double>(int, int, int, const double*, int64_t, double*, int64_t, hipStream_t);
template void launch_side_to_stack<float>(int, int, int, const double*, int64_t, float*, int64_t, hipStream_t);
template void launch_side_to_stack<bf16>(int, int, int, const double*, int64_t, bf16*, int64_t, hipStream_t);

}  // namespace isvd
