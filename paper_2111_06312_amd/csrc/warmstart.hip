// Learned warm start: per-node structural features, a 16 -> 128 -> 128 -> k
// MLP with GELU (FP32, MFMA), the subspace loss against target singular
// vectors, its backward pass and Adam.  The network's output replaces the
// first k columns of Algorithm 1's Gaussian start block.
//
// Loss (sign-, rotation- and scale-invariant; mean sin^2 of the principal
// angles between span(Z) and span(V)):
//   L = tr((Z^T Z)^-1 Z^T (I - V V^T) Z) / k = 1 - tr(G^-1 C C^T) / k,
//   G = Z^T Z, C = Z^T V,  dL/dZ = (2/k) (Z P P^T - V P^T),  P = G^-1 C.
#include <vector>

#include "operator.h"

struct isvd_warmstart {
  int k = 0;
  int64_t nparam = 0;
  isvd::DevBuf theta, grad, m1, m2;  // FP32 parameters, gradient, Adam moments
  int step = 0;
  // activations / temporaries for the last n
  isvd::DevBuf h1p, h1, h2p, h2, z, dz, dh, gtmp, small, work, f64buf, colsum;
  int64_t n_alloc = 0;
};

namespace isvd {

namespace {

constexpr int kIn = 16, kHid = 128;

// parameter offsets (floats) in theta: W1 16x128, b1, W2 128x128, b2, W3 128xk, b3
struct Layout {
  int64_t w1, b1, w2, b2, w3, b3, total;
  explicit Layout(int k) {
    w1 = 0;
    b1 = w1 + kIn * kHid;
    w2 = b1 + kHid;
    b2 = w2 + kHid * kHid;
    w3 = b2 + kHid;
    b3 = w3 + static_cast<int64_t>(kHid) * k;
    total = b3 + k;
  }
};

__device__ inline float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float x) {
  const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
  return cdf + x * pdf;
}

// C (M x N) = act(A) (M x K) * B (K x N) + bias (N);  act = identity or GELU.
// MFMA f32 16x16x4; block = 4 waves x 16 rows, columns in chunks of 16*TN.
template <int TN, bool GELU_A>
__global__ __launch_bounds__(256) void mlp_gemm_kernel(int64_t M, int N, int K, const float* A, int64_t lda,
                                                       const float* B, int64_t ldb, const float* bias, float* Cm,
                                                       int64_t ldc) {
  __shared__ float As[64][17];
  __shared__ float Bs[16][16 * TN];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * 64;
  const int col0 = blockIdx.y * 16 * TN;
  v4f acc[TN];
#pragma unroll
  for (int t = 0; t < TN; ++t) acc[t] = v4f{0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += 16) {
    __syncthreads();
    for (int f = threadIdx.x; f < 64 * 16; f += 256) {
      const int r = f >> 4, c = f & 15;
      const int64_t row = row0 + r;
      float v = 0.f;
      if (row < M && k0 + c < K) {
        v = A[row * lda + k0 + c];
        if (GELU_A) v = gelu_f(v);
      }
      As[r][c] = v;
    }
    for (int f = threadIdx.x; f < 16 * 16 * TN; f += 256) {
      const int r = f / (16 * TN), c = f % (16 * TN);
      Bs[r][c] = (k0 + r < K && col0 + c < N) ? B[static_cast<int64_t>(k0 + r) * ldb + col0 + c] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const float a = As[wave * 16 + li][kk * 4 + lk];
#pragma unroll
      for (int t = 0; t < TN; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, Bs[kk * 4 + lk][t * 16 + li], acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < TN; ++t) {
    const int col = col0 + t * 16 + li;
    if (col >= N) continue;
    const float bb = bias ? bias[col] : 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + wave * 16 + 4 * lk + r;
      if (row < M) Cm[row * ldc + col] = acc[t][r] + bb;
    }
  }
}

void mlp_gemm(int64_t M, int N, int K, const float* A, int64_t lda, bool gelu_a, const float* B, int64_t ldb,
              const float* bias, float* C, int64_t ldc, hipStream_t stream) {
  const unsigned gx = static_cast<unsigned>(ceil_div(M, 64));
  if (N <= 64) {
    const unsigned gy = static_cast<unsigned>(ceil_div(N, 64));
    if (gelu_a) hipLaunchKernelGGL((mlp_gemm_kernel<4, true>), dim3(gx, gy), dim3(256), 0, stream, M, N, K, A, lda, B, ldb, bias, C, ldc);
    else hipLaunchKernelGGL((mlp_gemm_kernel<4, false>), dim3(gx, gy), dim3(256), 0, stream, M, N, K, A, lda, B, ldb, bias, C, ldc);
  } else {
    const unsigned gy = static_cast<unsigned>(ceil_div(N, 128));
    if (gelu_a) hipLaunchKernelGGL((mlp_gemm_kernel<8, true>), dim3(gx, gy), dim3(256), 0, stream, M, N, K, A, lda, B, ldb, bias, C, ldc);
    else hipLaunchKernelGGL((mlp_gemm_kernel<8, false>), dim3(gx, gy), dim3(256), 0, stream, M, N, K, A, lda, B, ldb, bias, C, ldc);
  }
  ISVD_LAUNCH_CHECK();
}

// post = gelu(pre) (materialised for the weight gradients)
__global__ void gelu_kernel(int64_t total, const float* pre, float* post) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < total) post[i] = gelu_f(pre[i]);
}
// d *= gelu'(pre)
__global__ void gelu_back_kernel(int64_t total, const float* pre, float* d) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < total) d[i] *= gelu_grad_f(pre[i]);
}
// out (cols x rows) = in^T (rows x cols), FP32
__global__ void transpose_kernel(int rows, int cols, const float* in, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int r = i / cols, c = i % cols;
  out[static_cast<int64_t>(c) * rows + r] = in[i];
}
// FP64 grads -> FP32 slice of the flat gradient
__global__ void f64_to_f32_kernel(int64_t total, const double* in, float* out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < total) out[i] = static_cast<float>(in[i]);
}
// Adam (Kingma & Ba) on the flat parameter vector; bias corrections passed in.
__global__ void adam_kernel(int64_t total, float* theta, const float* g, float* m, float* v, float lr, float b1,
                            float b2, float eps, float c1, float c2, const int* breakdown) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total || *breakdown) return;   // no update from a step whose Cholesky failed
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- small FP64 helpers (k x k)

// P = Ginv C, PPt = P P^T, loss terms; one workgroup (k <= 512).
__global__ void loss_small_kernel(int k, const double* Ginv, const double* C, double* P, double* PPt,
                                  double* loss_out) {
  __shared__ double red[256];
  for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
    const int i = idx / k, j = idx % k;
    double s = 0.0;
    for (int t = 0; t < k; ++t) s += Ginv[i * k + t] * C[t * k + j];
    P[idx] = s;
  }
  __syncthreads();
  double tr = 0.0;
  for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
    const int i = idx / k, j = idx % k;
    double s = 0.0;
    for (int t = 0; t < k; ++t) s += P[i * k + t] * P[j * k + t];
    PPt[idx] = s;
    tr += P[idx] * C[idx];   // tr(P C^T) = sum_ij P_ij C_ij
  }
  red[threadIdx.x] = tr;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss_out = 1.0 - red[0] / k;
}

// B (2k x k, FP32) = (2/k) [P P^T ; -P^T]  (right operand of dZ = [Z | V] B)
__global__ void pack_dz_rhs_kernel(int k, const double* PPt, const double* P, float* B) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * k * k) return;
  const int r = idx / k, c = idx % k;
  const double s = 2.0 / k;
  const double v = r < k ? PPt[r * k + c] : -P[c * k + (r - k)];
  B[idx] = static_cast<float>(s * v);
}

// Ginv = Rinv Rinv^T from the inverse upper Cholesky factor (k x k, ld lp).
__global__ void spd_inverse_from_rinv_kernel(int k, int lp, const double* Rinv, double* Ginv) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= k * k) return;
  const int i = idx / k, j = idx % k;
  const int t0 = i > j ? i : j;
  double s = 0.0;
  for (int t = t0; t < k; ++t) s += Rinv[static_cast<int64_t>(i) * lp + t] * Rinv[static_cast<int64_t>(j) * lp + t];
  Ginv[idx] = s;
}

__global__ void identity_kernel(int n, int ld, double* A) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * ld) return;
  A[idx] = (idx / ld == idx % ld) ? 1.0 : 0.0;
}

// ---------------------------------------------------------------- features

// f[:, j] for one chain: x_{j} written into column col of the n x 16 FP64 block
__global__ void feature_finish_kernel(int64_t n, const double* raw, float* F, const double* mean, const double* sd,
                                      const int* ok) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n * kIn) return;
  const int c = static_cast<int>(i % kIn);
  F[i] = ok[c] ? static_cast<float>((log1p(raw[i]) - mean[c]) / sd[c]) : 0.f;
}

__global__ void feature_log_kernel(int64_t n, const double* raw, double* lg) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n * kIn) lg[i] = log1p(raw[i]);
}

// mean, population sd and the no-spread flag of each of the 16 columns (two passes, fixed order)
__global__ void feature_stats_kernel(int64_t n, const double* lg, double* mean, double* sd, int* ok) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += lg[i * kIn + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double mu = red[0] / static_cast<double>(n);
  __syncthreads();
  double q = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = lg[i * kIn + c] - mu;
    q += d * d;
  }
  red[threadIdx.x] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double sdv = sqrt(red[0] / static_cast<double>(n));
    mean[c] = mu;
    sd[c] = sdv;
    ok[c] = sdv > 1e-9 * (1.0 + fabs(mu)) ? 1 : 0;
  }
}

__global__ void fill_kernel(int64_t n, int64_t ld, double* x, const double* src, double value) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i * ld] = src ? src[i] : value;
}

// all entries finite?  flag stays 1 only if so
__global__ void finite_kernel(int64_t total, const float* z, int* flag) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < total && !isfinite(z[i])) *flag = 0;
}

template <typename T>
__global__ void omega_pack_kernel(int64_t n, int k, const float* Z, float scale, T* omega, int64_t ld) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n * k) return;
  const int64_t r = i / k;
  const int c = static_cast<int>(i % k);
  Elem<T>::store(omega + r * ld + c, static_cast<typename ComputeOf<T>::type>(scale * Z[i]));
}

unsigned nb(int64_t total) { return static_cast<unsigned>(ceil_div(total > 0 ? total : 1, 256)); }

void ensure_acts(isvd_warmstart* ws, int64_t n) {
  if (n <= ws->n_alloc) return;
  const size_t hid = static_cast<size_t>(n) * kHid * sizeof(float);
  ws->h1p.ensure(hid);
  ws->h1.ensure(hid);
  ws->h2p.ensure(hid);
  ws->h2.ensure(hid);
  ws->dh.ensure(hid);
  ws->gtmp.ensure(hid);
  ws->z.ensure(static_cast<size_t>(n) * ws->k * sizeof(float));
  ws->dz.ensure(static_cast<size_t>(n) * ws->k * sizeof(float));
  ws->n_alloc = n;
}

void forward(isvd_warmstart* ws, int64_t n, const float* F, float* Z, int64_t ldz, hipStream_t s) {
  const Layout L(ws->k);
  const float* th = ws->theta.as<float>();
  ensure_acts(ws, n);
  mlp_gemm(n, kHid, kIn, F, kIn, false, th + L.w1, kHid, th + L.b1, ws->h1p.as<float>(), kHid, s);
  mlp_gemm(n, kHid, kHid, ws->h1p.as<float>(), kHid, true, th + L.w2, kHid, th + L.b2, ws->h2p.as<float>(), kHid, s);
  mlp_gemm(n, ws->k, kHid, ws->h2p.as<float>(), kHid, true, th + L.w3, ws->k, th + L.b3, Z, ldz, s);
}

}  // namespace

// Structural features of the column-side nodes (see the header).
void ws_features(isvd_operator* op, float* F, hipStream_t s) {
  ISVD_CHECK(op->form == ISVD_FORM_NE, ISVD_E_INVALID, "features need an NE-form operator");
  const int64_t n = op->n;
  DevBuf raw, tmpa, tmpb, lg, stats;
  raw.ensure(static_cast<size_t>(n) * kIn * sizeof(double));
  lg.ensure(static_cast<size_t>(n) * kIn * sizeof(double));
  stats.ensure(64 * sizeof(double));
  double* R = raw.as<double>();
  const double* dinv = op->scale64.as<double>();
  // column 0: d;  columns 1..8: T^j d = D^-1 A x_{j-1} (rows of the forward CSR)
  hipLaunchKernelGGL(fill_kernel, dim3(nb(n)), dim3(256), 0, s, n, int64_t(kIn), R, op->deg.as<double>(), 0.0);
  ISVD_LAUNCH_CHECK();
  for (int j = 1; j <= 8; ++j) {
    SpmmPass p;
    p.n_rows = n; p.nnz = op->fwd.nnz; p.indptr = op->fwd.indptr; p.indices = op->fwd.indices; p.values = op->fwd.values;
    p.ncols = 1;
    p.src = R + (j - 1); p.ld_src = kIn;
    p.rowscale = dinv; p.a0 = 0.0; p.a1 = 1.0;
    p.out = R + j; p.ld_out = kIn;
    launch_spmm_pass<double>(p, s);
  }
  // columns 9..15: (T^T)^j 1 = A^T (D^-1 y_{j-1}), y_0 = 1
  hipLaunchKernelGGL(fill_kernel, dim3(nb(n)), dim3(256), 0, s, n, int64_t(1), lg.as<double>(), nullptr, 1.0);
  ISVD_LAUNCH_CHECK();
  for (int j = 1; j <= 7; ++j) {
    SpmmPass p;
    p.n_rows = n; p.nnz = op->bwd.nnz; p.indptr = op->bwd.indptr; p.indices = op->bwd.indices; p.values = op->bwd.values;
    p.ncols = 1;
    p.src = j == 1 ? lg.as<double>() : R + (8 + j - 1); p.ld_src = j == 1 ? 1 : kIn;
    p.colscale = dinv; p.cs_a = 1.0; p.cs_b = 0.0;
    p.a0 = 1.0;
    p.out = R + 8 + j; p.ld_out = kIn;
    launch_spmm_pass<double>(p, s);
  }
  hipLaunchKernelGGL(feature_log_kernel, dim3(nb(n * kIn)), dim3(256), 0, s, n, R, lg.as<double>());
  ISVD_LAUNCH_CHECK();
  double* mean = stats.as<double>();
  double* sd = mean + kIn;
  int* ok = reinterpret_cast<int*>(sd + kIn);
  hipLaunchKernelGGL(feature_stats_kernel, dim3(kIn), dim3(256), 0, s, n, lg.as<double>(), mean, sd, ok);
  ISVD_LAUNCH_CHECK();
  hipLaunchKernelGGL(feature_finish_kernel, dim3(nb(n * kIn)), dim3(256), 0, s, n, R, F, mean, sd, ok);
  ISVD_LAUNCH_CHECK();
  ISVD_HIP(hipStreamSynchronize(s));
}

void ws_forward(isvd_warmstart* ws, int64_t n, const float* F, float* Z, int64_t ldz, hipStream_t s) {
  forward(ws, n, F, Z, ldz, s);
}

// Loss and gradient for one graph; optional Adam step.
void ws_train_step(isvd_warmstart* ws, int64_t n, const float* F, const float* V, int64_t ldv, double lr,
                   double* loss_out, float* grad_host, hipStream_t s) {
  const int k = ws->k;
  const Layout L(k);
  ensure_acts(ws, n);
  float* Z = ws->z.as<float>();
  forward(ws, n, F, Z, k, s);
  // G = Z^T Z, C = Z^T V (FP64)
  const int lp = pad16(k);
  ws->small.ensure(static_cast<size_t>(12) * lp * lp * sizeof(double) + 64);
  double* G = ws->small.as<double>();
  double* C = G + static_cast<int64_t>(lp) * lp;
  double* R64 = C + static_cast<int64_t>(lp) * lp;
  double* Rinv = R64 + static_cast<int64_t>(lp) * lp;
  double* Rc = Rinv + static_cast<int64_t>(lp) * lp;
  double* Dc = Rc + static_cast<int64_t>(lp) * lp;
  double* Ginv = Dc + static_cast<int64_t>(lp) * 16;
  double* P = Ginv + static_cast<int64_t>(lp) * lp;
  double* PPt = P + static_cast<int64_t>(lp) * lp;
  double* loss_d = PPt + static_cast<int64_t>(lp) * lp;
  int* flag = reinterpret_cast<int*>(loss_d + 2);
  const size_t gw = gram_workspace_doubles(n, k, k);
  size_t wneed = gw;
  const size_t g2 = gram_workspace_doubles(n, kHid, kHid > k ? kHid : k);
  const size_t g3 = gram_workspace_doubles(n, kIn, kHid);
  const size_t g4 = gram_workspace_doubles(n, kHid, k);   // each Gram shape below sizes its own slices
  wneed = wneed > g2 ? wneed : g2;
  wneed = wneed > g3 ? wneed : g3;
  wneed = wneed > g4 ? wneed : g4;
  ws->work.ensure(wneed * sizeof(double));
  double* work = ws->work.as<double>();
  launch_gram<float>(n, k, k, Z, k, Z, k, true, G, k, work, s);
  launch_gram2<float, float>(n, k, k, Z, k, V, ldv, C, k, work, s);
  // G^-1 = R^-1 R^-T  (R: Cholesky factor; R^-1 by the tall solve applied to I)
  launch_cholesky<double>(k, G, k, 0.0, 1e-14, R64, Rc, Dc, flag, 0, s);
  hipLaunchKernelGGL(identity_kernel, dim3(nb(static_cast<int64_t>(k) * lp)), dim3(256), 0, s, k, lp, Rinv);
  ISVD_LAUNCH_CHECK();
  launch_trsm_tall<double>(k, k, Rinv, lp, Rc, Dc, nullptr, nullptr, s);
  hipLaunchKernelGGL(spd_inverse_from_rinv_kernel, dim3(nb(static_cast<int64_t>(k) * k)), dim3(256), 0, s, k, lp,
                     Rinv, Ginv);
  ISVD_LAUNCH_CHECK();
  hipLaunchKernelGGL(loss_small_kernel, dim3(1), dim3(256), 0, s, k, Ginv, C, P, PPt, loss_d);
  ISVD_LAUNCH_CHECK();
  // dZ = [Z | V] (2/k) [P P^T ; -P^T]
  ws->f64buf.ensure(static_cast<size_t>(2) * k * k * sizeof(float) + static_cast<size_t>(kHid) * kHid * sizeof(float));
  float* Bdz = ws->f64buf.as<float>();
  hipLaunchKernelGGL(pack_dz_rhs_kernel, dim3(nb(2 * k * k)), dim3(256), 0, s, k, PPt, P, Bdz);
  ISVD_LAUNCH_CHECK();
  float* dZ = ws->dz.as<float>();
  launch_gemm_tall<float>(n, k, k, Z, k, k, V, ldv, Bdz, k, dZ, k, 1.0, 0.0, GemmEpi::Store, nullptr, nullptr, s);
  // backward through the network
  float* grad = ws->grad.as<float>();
  const float* th = ws->theta.as<float>();
  DevBuf g64, wt;
  g64.ensure(static_cast<size_t>(kHid) * (kHid > k ? kHid : k) * sizeof(double));
  wt.ensure(static_cast<size_t>(kHid) * (kHid > k ? kHid : k) * sizeof(float));
  double* gd = g64.as<double>();
  float* h1 = ws->h1.as<float>();
  float* h2 = ws->h2.as<float>();
  const int64_t nh = n * kHid;
  hipLaunchKernelGGL(gelu_kernel, dim3(nb(nh)), dim3(256), 0, s, nh, ws->h1p.as<float>(), h1);
  hipLaunchKernelGGL(gelu_kernel, dim3(nb(nh)), dim3(256), 0, s, nh, ws->h2p.as<float>(), h2);
  ISVD_LAUNCH_CHECK();
  // column sums: result (<= 512 doubles) then the colsum partials
  const int wmax = kHid > k ? kHid : k;
  ws->colsum.ensure((static_cast<size_t>(kColsumBlocks) * wmax + 512) * sizeof(double));
  double* cs = ws->colsum.as<double>();
  // layer 3: dW3 = H2^T dZ, db3 = 1^T dZ, dH2 = dZ W3^T, then * gelu'(H2p)
  launch_gram2<float, float>(n, kHid, k, h2, kHid, dZ, k, gd, k, work, s);
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(nb(kHid * k)), dim3(256), 0, s, int64_t(kHid) * k, gd, grad + L.w3);
  launch_colsum<float>(n, k, dZ, k, cs + 512, cs, s);
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(nb(k)), dim3(256), 0, s, int64_t(k), cs, grad + L.b3);
  hipLaunchKernelGGL(transpose_kernel, dim3(nb(kHid * k)), dim3(256), 0, s, kHid, k, th + L.w3, wt.as<float>());
  ISVD_LAUNCH_CHECK();
  float* dH = ws->dh.as<float>();
  mlp_gemm(n, kHid, k, dZ, k, false, wt.as<float>(), kHid, nullptr, dH, kHid, s);
  hipLaunchKernelGGL(gelu_back_kernel, dim3(nb(nh)), dim3(256), 0, s, nh, ws->h2p.as<float>(), dH);
  ISVD_LAUNCH_CHECK();
  // layer 2: dW2 = H1^T dH2p, db2, dH1 = dH2p W2^T, * gelu'(H1p)
  launch_gram2<float, float>(n, kHid, kHid, h1, kHid, dH, kHid, gd, kHid, work, s);
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(nb(kHid * kHid)), dim3(256), 0, s, int64_t(kHid) * kHid, gd, grad + L.w2);
  launch_colsum<float>(n, kHid, dH, kHid, cs + 512, cs, s);
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(nb(kHid)), dim3(256), 0, s, int64_t(kHid), cs, grad + L.b2);
  hipLaunchKernelGGL(transpose_kernel, dim3(nb(kHid * kHid)), dim3(256), 0, s, kHid, kHid, th + L.w2, wt.as<float>());
  ISVD_LAUNCH_CHECK();
  float* dH1 = ws->gtmp.as<float>();
  mlp_gemm(n, kHid, kHid, dH, kHid, false, wt.as<float>(), kHid, nullptr, dH1, kHid, s);
  hipLaunchKernelGGL(gelu_back_kernel, dim3(nb(nh)), dim3(256), 0, s, nh, ws->h1p.as<float>(), dH1);
  ISVD_LAUNCH_CHECK();
  // layer 1: dW1 = F^T dH1p, db1
  launch_gram2<float, float>(n, kIn, kHid, F, kIn, dH1, kHid, gd, kHid, work, s);
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(nb(kIn * kHid)), dim3(256), 0, s, int64_t(kIn) * kHid, gd, grad + L.w1);
  launch_colsum<float>(n, kHid, dH1, kHid, cs + 512, cs, s);
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(nb(kHid)), dim3(256), 0, s, int64_t(kHid), cs, grad + L.b1);
  ISVD_LAUNCH_CHECK();
  if (lr > 0.0) {
    ws->step++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, static_cast<float>(ws->step));
    const float c2 = 1.f - powf(b2, static_cast<float>(ws->step));
    hipLaunchKernelGGL(adam_kernel, dim3(nb(L.total)), dim3(256), 0, s, L.total, ws->theta.as<float>(), grad,
                       ws->m1.as<float>(), ws->m2.as<float>(), static_cast<float>(lr), b1, b2, 1e-8f, c1, c2, flag);
    ISVD_LAUNCH_CHECK();
  }
  int fl = 0;
  ISVD_HIP(hipMemcpyAsync(loss_out, loss_d, sizeof(double), hipMemcpyDeviceToHost, s));
  ISVD_HIP(hipMemcpyAsync(&fl, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  if (grad_host) ISVD_HIP(hipMemcpyAsync(grad_host, grad, L.total * sizeof(float), hipMemcpyDeviceToHost, s));
  ISVD_HIP(hipStreamSynchronize(s));
  ISVD_CHECK(fl == 0, ISVD_E_NOT_SPD, "network output is rank deficient (Z^T Z not positive definite)");
}

// Start block [MLP(F) | Gaussian] with fallback to all-Gaussian.
void ws_omega(isvd_warmstart* ws, isvd_operator* op, const float* F, int p, uint64_t seed, void* omega,
              int64_t ld, int* used_fallback, hipStream_t s) {
  const int64_t n = op->cols;
  const int k = ws->k;
  ensure_acts(ws, n);
  float* Z = ws->z.as<float>();
  forward(ws, n, F, Z, k, s);
  DevBuf fl;
  fl.ensure(sizeof(int) * 2);
  int one = 1;
  ISVD_HIP(hipMemcpyAsync(fl.p, &one, sizeof(int), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(finite_kernel, dim3(nb(n * k)), dim3(256), 0, s, n * k, Z, fl.as<int>());
  ISVD_LAUNCH_CHECK();
  int finite = 0;
  ISVD_HIP(hipMemcpyAsync(&finite, fl.p, sizeof(int), hipMemcpyDeviceToHost, s));
  ISVD_HIP(hipStreamSynchronize(s));
  bool ok = finite != 0;
  if (ok) {
    // full column rank: Cholesky of Z^T Z must succeed; then one Cholesky QR
    // pass, Z <- Z R^-1, hands Algorithm 1 orthonormal columns instead of the
    // raw (possibly ill-conditioned) network output
    const int lp = pad16(k);
    DevBuf G, R64, Rc, Dc, cf, work;
    G.ensure(static_cast<size_t>(k) * k * sizeof(double));
    R64.ensure(static_cast<size_t>(lp) * lp * sizeof(double));
    Rc.ensure(static_cast<size_t>(lp) * lp * sizeof(float));
    Dc.ensure(static_cast<size_t>(lp) * 16 * sizeof(float));
    cf.ensure(sizeof(int));
    work.ensure(gram_workspace_doubles(n, k, k) * sizeof(double));
    launch_gram<float>(n, k, k, Z, k, Z, k, true, G.as<double>(), k, work.as<double>(), s);
    launch_cholesky<float>(k, G.as<double>(), k, 0.0, 1e-12, R64.as<double>(), Rc.as<float>(), Dc.as<float>(),
                           cf.as<int>(), 0, s);
    int bad = 0;
    ISVD_HIP(hipMemcpyAsync(&bad, cf.p, sizeof(int), hipMemcpyDeviceToHost, s));
    ISVD_HIP(hipStreamSynchronize(s));
    ok = bad == 0;
    if (ok) launch_trsm_tall<float>(n, k, Z, k, Rc.as<float>(), Dc.as<float>(), nullptr, nullptr, s);
    ISVD_HIP(hipStreamSynchronize(s));   // the factors are freed on leaving this block
  }
  // orthonormal columns scaled to the norm of the Gaussian columns beside them
  const float zscale = std::sqrt(static_cast<float>(n));
  const int l = k + p;
  switch (op->prec) {
    case ISVD_FP64: {
      double* o = static_cast<double*>(omega);
      launch_gaussian<double>(n, l, seed, o, ld, s);
      if (ok) hipLaunchKernelGGL(omega_pack_kernel<double>, dim3(nb(n * k)), dim3(256), 0, s, n, k, Z, zscale, o, ld);
      break;
    }
    case ISVD_FP32: {
      float* o = static_cast<float*>(omega);
      launch_gaussian<float>(n, l, seed, o, ld, s);
      if (ok) hipLaunchKernelGGL(omega_pack_kernel<float>, dim3(nb(n * k)), dim3(256), 0, s, n, k, Z, zscale, o, ld);
      break;
    }
    default: {
      bf16* o = static_cast<bf16*>(omega);
      launch_gaussian<bf16>(n, l, seed, o, ld, s);
      if (ok) hipLaunchKernelGGL(omega_pack_kernel<bf16>, dim3(nb(n * k)), dim3(256), 0, s, n, k, Z, zscale, o, ld);
      break;
    }
  }
  ISVD_LAUNCH_CHECK();
  ISVD_HIP(hipStreamSynchronize(s));
  if (used_fallback) *used_fallback = ok ? 0 : 1;
}

void ws_init(isvd_warmstart* ws, int k, uint64_t seed) {
  const Layout L(k);
  ws->k = k;
  ws->nparam = L.total;
  const size_t bytes = L.total * sizeof(float);
  ws->theta.ensure(bytes);
  ws->grad.ensure(bytes);
  ws->m1.ensure(bytes);
  ws->m2.ensure(bytes);
  ISVD_HIP(hipMemset(ws->theta.p, 0, bytes));
  ISVD_HIP(hipMemset(ws->grad.p, 0, bytes));
  ISVD_HIP(hipMemset(ws->m1.p, 0, bytes));
  ISVD_HIP(hipMemset(ws->m2.p, 0, bytes));
  // weights N(0, 1/fan_in) from the device Philox stream (one seed per matrix), biases 0
  const int64_t fan[3] = {kIn, kHid, kHid};
  const int64_t off[3] = {L.w1, L.w2, L.w3};
  const int64_t cols[3] = {kHid, kHid, k};
  for (int i = 0; i < 3; ++i) {
    float* w = ws->theta.as<float>() + off[i];
    launch_gaussian<float>(fan[i], cols[i], seed + static_cast<uint64_t>(i), w, cols[i], nullptr);
    std::vector<float> h(static_cast<size_t>(fan[i] * cols[i]));
    ISVD_HIP(hipMemcpy(h.data(), w, h.size() * sizeof(float), hipMemcpyDeviceToHost));
    const float sc = 1.0f / std::sqrt(static_cast<float>(fan[i]));
    for (float& v : h) v *= sc;
    ISVD_HIP(hipMemcpy(w, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
  }
}

}  // namespace isvd

using namespace isvd;

namespace isvd {
template <typename F>
isvd_status ws_guarded(F&& f) {
  try {
    set_last_error("");
    return f();
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return ISVD_E_INVALID;
  }
}
}  // namespace isvd

extern "C" {

isvd_status isvd_ws_features(isvd_operator* op, float* F, void* stream) {
  return ws_guarded([&]() -> isvd_status {
    ISVD_CHECK(op && F, ISVD_E_INVALID, "null argument");
    ws_features(op, F, static_cast<hipStream_t>(stream));
    return ISVD_OK;
  });
}

isvd_status isvd_ws_create(int k, uint64_t seed, isvd_warmstart** out) {
  return ws_guarded([&]() -> isvd_status {
    ISVD_CHECK(out && k >= 1 && k <= 512, ISVD_E_INVALID, "need 1 <= k <= 512");
    *out = nullptr;
    auto* ws = new isvd_warmstart();
    try {
      ws_init(ws, k, seed);
    } catch (...) {
      delete ws;
      throw;
    }
    *out = ws;
    return ISVD_OK;
  });
}

void isvd_ws_destroy(isvd_warmstart* ws) {
  if (!ws) return;
  (void)hipDeviceSynchronize();
  delete ws;
}

int64_t isvd_ws_num_params(const isvd_warmstart* ws) { return ws ? ws->nparam : 0; }

isvd_status isvd_ws_get_params(const isvd_warmstart* ws, float* host_out) {
  return ws_guarded([&]() -> isvd_status {
    ISVD_CHECK(ws && host_out, ISVD_E_INVALID, "null argument");
    ISVD_HIP(hipMemcpy(host_out, ws->theta.p, ws->nparam * sizeof(float), hipMemcpyDeviceToHost));
    return ISVD_OK;
  });
}

isvd_status isvd_ws_set_params(isvd_warmstart* ws, const float* host_in) {
  return ws_guarded([&]() -> isvd_status {
    ISVD_CHECK(ws && host_in, ISVD_E_INVALID, "null argument");
    ISVD_HIP(hipMemcpy(ws->theta.p, host_in, ws->nparam * sizeof(float), hipMemcpyHostToDevice));
    return ISVD_OK;
  });
}

isvd_status isvd_ws_forward(isvd_warmstart* ws, int64_t n, const float* F, float* Z, int64_t ldz, void* stream) {
  return ws_guarded([&]() -> isvd_status {
    ISVD_CHECK(ws && F && Z && n >= 1 && ldz >= ws->k, ISVD_E_INVALID, "bad forward arguments");
    ws_forward(ws, n, F, Z, ldz, static_cast<hipStream_t>(stream));
    return ISVD_OK;
  });
}

isvd_status isvd_ws_train_step(isvd_warmstart* ws, int64_t n, const float* F, const float* V, int64_t ldv,
                               double lr, double* loss_out, float* grad_out, void* stream) {
  return ws_guarded([&]() -> isvd_status {
    ISVD_CHECK(ws && F && V && loss_out && n >= ws->k && ldv >= ws->k, ISVD_E_INVALID, "bad train-step arguments");
    ws_train_step(ws, n, F, V, ldv, lr, loss_out, grad_out, static_cast<hipStream_t>(stream));
    return ISVD_OK;
  });
}

isvd_status isvd_ws_omega(isvd_warmstart* ws, isvd_operator* op, const float* F, int p, uint64_t seed, void* omega,
                          int64_t ld_omega, int* used_fallback, void* stream) {
  return ws_guarded([&]() -> isvd_status {
    ISVD_CHECK(ws && op && F && omega && p >= 0 && ld_omega >= ws->k + p, ISVD_E_INVALID, "bad omega arguments");
    ISVD_CHECK(op->form == ISVD_FORM_NE, ISVD_E_INVALID, "warm start needs an NE-form operator");
    ws_omega(ws, op, F, p, seed, omega, ld_omega, used_fallback, static_cast<hipStream_t>(stream));
    return ISVD_OK;
  });
}

}  // extern "C"
