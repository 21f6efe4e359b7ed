// Closed-form learners on a rank-k SVD (Section 3): node embeddings and pair
// scores (Eq. 5), and the least-norm linear model W* = V S^+ U^T Y (Eq. 8),
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

// out[i][t] = in[i][t] * sqrt(s_t) for two matrices in one launch (blocks
// below `split` take the first).  A thread owns VW consecutive columns of
// one row: `kq` threads cover a row (k = VW kq), a block covers 256 / kq
// rows per step and walks its share of rows with a stride.
template <typename T, int VW>
__global__ __launch_bounds__(256) void embed_kernel(int k, int kq, const double* s, unsigned split, int64_t rows0,
                                                     const T* in0, int64_t ldi0, T* out0, int64_t ldo0, int64_t rows1,
                                                     const T* in1, int64_t ldi1, T* out1, int64_t ldo1) {
  const bool second = blockIdx.x >= split;
  const int64_t rows = second ? rows1 : rows0;
  const T* in = second ? in1 : in0;
  T* out = second ? out1 : out0;
  const int64_t ldi = second ? ldi1 : ldi0, ldo = second ? ldo1 : ldo0;
  const unsigned blk = second ? blockIdx.x - split : blockIdx.x;
  const unsigned nblk = second ? gridDim.x - split : split;
  const int per = 256 / kq;
  const int cq = static_cast<int>(threadIdx.x) % kq, ro = static_cast<int>(threadIdx.x) / kq;
  if (ro >= per) return;
  const int c = VW * cq;
  double r[VW];
#pragma unroll
  for (int e = 0; e < VW; ++e) r[e] = c + e < k ? sqrt(s[c + e]) : 0.0;
  for (int64_t i = static_cast<int64_t>(blk) * per + ro; i < rows; i += static_cast<int64_t>(nblk) * per) {
    const T* src = in + i * ldi + c;
    T* dst = out + i * ldo + c;
    if constexpr (VW == 4 && std::is_same<T, float>::value) {
      const float4 v = *reinterpret_cast<const float4*>(src);
      *reinterpret_cast<float4*>(dst) = make_float4(static_cast<float>(v.x * r[0]), static_cast<float>(v.y * r[1]),
                                                    static_cast<float>(v.z * r[2]), static_cast<float>(v.w * r[3]));
    } else if constexpr (VW == 2 && std::is_same<T, double>::value) {
      const double2 v = *reinterpret_cast<const double2*>(src);
      *reinterpret_cast<double2*>(dst) = make_double2(v.x * r[0], v.y * r[1]);
    } else {
#pragma unroll
      for (int e = 0; e < VW; ++e)
        if (c + e < k) dst[e] = static_cast<T>(static_cast<double>(src[e]) * r[e]);
    }
  }
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

// dst0[r] = src0[rows[r]] (cols0 columns) and dst1[r] = src1[rows[r]]
// (cols1 columns): one wave per gathered row.  Rows out of range give zeros
// and raise the flag.
template <typename T>
__global__ __launch_bounds__(256) void gather_rows_kernel(int64_t nsub, const int64_t* rows, int64_t nsrc, int cols0,
                                                           const T* src0, int64_t lds0, T* dst0, int64_t ldd0,
                                                           int cols1, const T* src1, int64_t lds1, T* dst1,
                                                           int64_t ldd1, int* bad) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; r < nsub;
       r += (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6) {
    const int64_t sr = rows[r];
    const bool ok = sr >= 0 && sr < nsrc;
    if (!ok && lane == 0) atomicOr(bad, 1);
    const T* a = src0 + (ok ? sr : 0) * lds0;
    T* da = dst0 + r * ldd0;
    for (int c = lane; c < cols0; c += 64) da[c] = ok ? a[c] : T(0);
    const T* b = src1 + (ok ? sr : 0) * lds1;
    T* db = dst1 + r * ldd1;
    for (int c = lane; c < cols1; c += 64) db[c] = ok ? b[c] : T(0);
  }
}

// W[j][y] = sum_t V[j][t] s^+_t T[t][y] (FP64), s^+_t = 1/s_t for s_t > rcond
// max(s), else 0.  One 64-lane block per row j and 64 label columns
// (blockIdx.y); T stays in L2 across the blocks.
template <typename T>
__global__ __launch_bounds__(64) void nc_apply_kernel(int64_t rows, int k, int ny, const T* V, int64_t ldv,
                                                       const double* s, double rcond, const double* Tm, int64_t ldt,
                                                       double* W, int64_t ldw) {
  __shared__ double sp[1024];
  const int lane = threadIdx.x;
  double m = 0.0;
  for (int t = lane; t < k; t += 64) m = fmax(m, s[t]);
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  const double cut = rcond * m;
  for (int t = lane; t < k; t += 64) sp[t] = s[t] > cut ? 1.0 / s[t] : 0.0;
  __syncthreads();
  const int y = static_cast<int>(blockIdx.y) * 64 + lane;
  const int yc = y < ny ? y : ny - 1;
  for (int64_t j = blockIdx.x; j < rows; j += gridDim.x) {
    const T* vr = V + j * ldv;
    const double* tc = Tm + yc;
    double acc0 = 0.0, acc1 = 0.0;
    int t = 0;
    for (; t + 1 < k; t += 2) {
      acc0 += static_cast<double>(vr[t]) * sp[t] * tc[static_cast<int64_t>(t) * ldt];
      acc1 += static_cast<double>(vr[t + 1]) * sp[t + 1] * tc[static_cast<int64_t>(t + 1) * ldt];
    }
    if (t < k) acc0 += static_cast<double>(vr[t]) * sp[t] * tc[static_cast<int64_t>(t) * ldt];
    if (y < ny) W[j * ldw + y] = acc0 + acc1;
  }
}

}  // namespace

template <typename T>
void launch_ne_embed(int k, const double* s, int64_t rows0, const T* in0, int64_t ldi0, T* out0, int64_t ldo0,
                     int64_t rows1, const T* in1, int64_t ldi1, T* out1, int64_t ldo1, hipStream_t stream) {
  ISVD_CHECK(k >= 1 && k <= 1024, ISVD_E_INVALID, "embeddings: k out of range");
  if (rows0 + rows1 == 0) return;
  constexpr int VV = std::is_same<T, float>::value ? 4 : 2;
  auto aligned = [&](const void* p, int64_t ld) {
    return reinterpret_cast<uintptr_t>(p) % (VV * sizeof(T)) == 0 && ld % VV == 0;
  };
  const bool vec = k % VV == 0 && (rows0 == 0 || (aligned(in0, ldi0) && aligned(out0, ldo0))) &&
                   (rows1 == 0 || (aligned(in1, ldi1) && aligned(out1, ldo1)));
  const int vw = vec ? VV : 1;
  const int kq = static_cast<int>(ceil_div(k, vw));
  const int per = kq <= 256 ? 256 / kq : 0;
  ISVD_CHECK(per > 0, ISVD_E_INVALID, "embeddings: k too large for one row per block");
  // about 4 row steps per block; both matrices in one grid
  const int64_t b0 = std::min<int64_t>(ceil_div(rows0, 4 * per), 1 << 20);
  const int64_t b1 = std::min<int64_t>(ceil_div(rows1, 4 * per), 1 << 20);
  const dim3 grid(static_cast<unsigned>(b0 + b1));
  const unsigned split = static_cast<unsigned>(b0);
  if (vec)
    hipLaunchKernelGGL((embed_kernel<T, VV>), grid, dim3(256), 0, stream, k, kq, s, split, rows0, in0, ldi0, out0,
                       ldo0, rows1, in1, ldi1, out1, ldo1);
  else
    hipLaunchKernelGGL((embed_kernel<T, 1>), grid, dim3(256), 0, stream, k, kq, s, split, rows0, in0, ldi0, out0,
                       ldo0, rows1, in1, ldi1, out1, ldo1);
  ISVD_LAUNCH_CHECK();
}
template void launch_ne_embed<float>(int, const double*, int64_t, const float*, int64_t, float*, int64_t, int64_t,
                                     const float*, int64_t, float*, int64_t, hipStream_t);
template void launch_ne_embed<double>(int, const double*, int64_t, const double*, int64_t, double*, int64_t, int64_t,
                                      const double*, int64_t, double*, int64_t, hipStream_t);

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
void launch_gather_rows(int64_t nsub, const int64_t* rows, int64_t nsrc, int cols0, const T* src0, int64_t lds0,
                        T* dst0, int64_t ldd0, int cols1, const T* src1, int64_t lds1, T* dst1, int64_t ldd1, int* bad,
                        hipStream_t stream) {
  if (nsub == 0) return;
  const int64_t blocks = std::min<int64_t>(ceil_div(nsub, 4), 8192);
  hipLaunchKernelGGL(gather_rows_kernel<T>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, nsub, rows,
                     nsrc, cols0, src0, lds0, dst0, ldd0, cols1, src1, lds1, dst1, ldd1, bad);
  ISVD_LAUNCH_CHECK();
}
template void launch_gather_rows<float>(int64_t, const int64_t*, int64_t, int, const float*, int64_t, float*, int64_t,
                                        int, const float*, int64_t, float*, int64_t, int*, hipStream_t);
template void launch_gather_rows<double>(int64_t, const int64_t*, int64_t, int, const double*, int64_t, double*,
                                         int64_t, int, const double*, int64_t, double*, int64_t, int*, hipStream_t);

template <typename T>
void launch_nc_apply(int64_t rows, int k, int ny, const T* V, int64_t ldv, const double* s, double rcond,
                     const double* Tm, int64_t ldt, double* W, int64_t ldw, hipStream_t stream) {
  ISVD_CHECK(k >= 1 && k <= 1024, ISVD_E_INVALID, "nc fit: k out of range");
  if (rows == 0 || ny == 0) return;
  const int64_t ychunks = ceil_div(ny, 64);
  ISVD_CHECK(ychunks <= 65535, ISVD_E_INVALID, "nc fit: too many label columns");
  const int64_t blocks = std::min<int64_t>(rows, 16384);
  hipLaunchKernelGGL(nc_apply_kernel<T>, dim3(static_cast<unsigned>(blocks), static_cast<unsigned>(ychunks)),
                     dim3(64), 0, stream, rows, k, ny, V, ldv, s, rcond, Tm, ldt, W, ldw);
  ISVD_LAUNCH_CHECK();
}
template void launch_nc_apply<float>(int64_t, int, int, const float*, int64_t, const double*, double, const double*,
                                     int64_t, double*, int64_t, hipStream_t);
template void launch_nc_apply<double>(int64_t, int, int, const double*, int64_t, const double*, double,
                                      const double*, int64_t, double*, int64_t, hipStream_t);

}  // namespace isvd
