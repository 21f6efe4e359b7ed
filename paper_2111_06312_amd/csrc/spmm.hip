// Fused CSR x tall-skinny pass (see spmm.h) and FP64 column sums.
//
// Light rows: a group of G lanes (G in {8, 16, 32, 64}) owns one output row
// and all its columns; each lane holds NV 16-byte chunks of the row (or NV
// single elements when the block is not 16-byte aligned).  The group
// prefetches up to G column indices with one coalesced load, then
// broadcasts them lane to lane and keeps U independent row gathers in
// flight.  Rows longer than heavy_threshold ("hubs" of power-law graphs)
// are taken by whole workgroups: four waves stride over the row's
// nonzeros and combine their partial rows through LDS in a fixed order.
#include "spmm.h"

namespace isvd {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
// Gathers in flight per lane group.  Loads stay in their 16-byte storage form
// until their FMAs, so the registers (and the occupancy) do not grow with
// the unpacked width; deeper unrolling measured slower (fewer waves per SIMD).
constexpr int kUnroll = 4;

// The row-wise streams of a pass (column ids, edge values, the added block
// and the outputs) are touched once: their loads and stores are marked
// non-temporal, so that they displace fewer of the gathered rows from the
// caches (measured: 1.6% shorter FP32 passes on the 2,000,000-node graph).
typedef float v4f_stream __attribute__((ext_vector_type(4)));
typedef unsigned v4u_stream __attribute__((ext_vector_type(4)));
template <typename V> __device__ inline V stream_load(const V* p) { return __builtin_nontemporal_load(p); }
template <typename V> __device__ inline void stream_store(V v, V* p) { __builtin_nontemporal_store(v, p); }

// 16-byte chunk (VEC) or single-element access to a storage row.
template <typename T, typename C, bool VEC> struct Chunk;

template <typename T, typename C> struct Chunk<T, C, false> {
  static constexpr int N = 1;
  using Raw = C;
  __device__ static inline Raw load_raw(const T* p) { return static_cast<C>(Elem<T>::load(p)); }
  __device__ static inline void unpack(const Raw& r, C (&x)[N]) { x[0] = r; }
  __device__ static inline void load(const T* p, C (&x)[N]) { x[0] = static_cast<C>(Elem<T>::load(p)); }
  __device__ static inline void load_stream(const T* p, C (&x)[N]) { load(p, x); }
  __device__ static inline void store(T* p, const C (&x)[N], int valid) {
    if (valid > 0) Elem<T>::store(p, x[0]);
  }
};

template <> struct Chunk<float, float, true> {
  static constexpr int N = 4;
  using Raw = float4;
  __device__ static inline Raw load_raw(const float* p) { return *reinterpret_cast<const float4*>(p); }
  __device__ static inline void unpack(const Raw& v, float (&x)[N]) {
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
  }
  __device__ static inline void load(const float* p, float (&x)[N]) {
    float4 v = *reinterpret_cast<const float4*>(p);
    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
  }
  __device__ static inline void load_stream(const float* p, float (&x)[N]) {
    const v4f_stream v = stream_load(reinterpret_cast<const v4f_stream*>(p));
    x[0] = v[0]; x[1] = v[1]; x[2] = v[2]; x[3] = v[3];
  }
  __device__ static inline void store(float* p, const float (&x)[N], int valid) {
    if (valid >= N) {
      stream_store(v4f_stream{x[0], x[1], x[2], x[3]}, reinterpret_cast<v4f_stream*>(p));
    } else {
      for (int t = 0; t < valid; ++t) p[t] = x[t];
    }
  }
};

template <> struct Chunk<double, double, true> {
  static constexpr int N = 2;
  using Raw = double2;
  __device__ static inline Raw load_raw(const double* p) { return *reinterpret_cast<const double2*>(p); }
  __device__ static inline void unpack(const Raw& v, double (&x)[N]) { x[0] = v.x; x[1] = v.y; }
  __device__ static inline void load(const double* p, double (&x)[N]) {
    double2 v = *reinterpret_cast<const double2*>(p);
    x[0] = v.x; x[1] = v.y;
  }
  __device__ static inline void load_stream(const double* p, double (&x)[N]) { load(p, x); }
  __device__ static inline void store(double* p, const double (&x)[N], int valid) {
    if (valid >= N) {
      *reinterpret_cast<double2*>(p) = make_double2(x[0], x[1]);
    } else if (valid > 0) {
      p[0] = x[0];
    }
  }
};

template <> struct Chunk<bf16, float, true> {
  static constexpr int N = 8;
  using Raw = uint4;
  __device__ static inline Raw load_raw(const bf16* p) { return *reinterpret_cast<const uint4*>(p); }
  __device__ static inline void unpack(const Raw& v, float (&x)[N]) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      x[2 * t] = bf16_to_float(static_cast<uint16_t>(w[t] & 0xffffu));
      x[2 * t + 1] = bf16_to_float(static_cast<uint16_t>(w[t] >> 16));
    }
  }
  __device__ static inline void load(const bf16* p, float (&x)[N]) { unpack(load_raw(p), x); }
  __device__ static inline void load_stream(const bf16* p, float (&x)[N]) {
    const v4u_stream v = stream_load(reinterpret_cast<const v4u_stream*>(p));
    unpack(make_uint4(v[0], v[1], v[2], v[3]), x);
  }
  __device__ static inline void store(bf16* p, const float (&x)[N], int valid) {
    if (valid >= N) {
      uint32_t w[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) w[t] = float2_to_bf16x2(x[2 * t], x[2 * t + 1]);
      stream_store(v4u_stream{w[0], w[1], w[2], w[3]}, reinterpret_cast<v4u_stream*>(p));
    } else {
      for (int t = 0; t < valid; ++t) p[t].bits = float_to_bf16(x[t]);
    }
  }
};

template <int G>
__device__ inline int bcast_i(int v, int src) {
  if constexpr (G == 64) return __builtin_amdgcn_readlane(v, src);
  else return __shfl(v, src, 64);
}
template <int G>
__device__ inline float bcast_f(float v, int src) {
  if constexpr (G == 64) return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
  else return __shfl(v, src, 64);
}
template <int G>
__device__ inline double bcast_f(double v, int src) {
  if constexpr (G == 64) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffll), src);
    int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), src);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
  } else {
    return __shfl(v, src, 64);
  }
}

// acc += sum over nonzeros base, base+step, ... (batches of G) of g * Src row.
// gl: lane within group, gbase: first lane of the group, lanes own chunks gl + G*m.
template <typename T, typename C, int G, int NV, bool VEC>
__device__ inline void accumulate(const SpmmPass& p, int64_t beg, int64_t end, int64_t step, int gl,
                                  int gbase, int nchunks, C (&acc)[NV][Chunk<T, C, VEC>::N]) {
  using CK = Chunk<T, C, VEC>;
  constexpr int EPC = CK::N;
  constexpr int U = kUnroll;
  const T* src = static_cast<const T*>(p.src);
  const int64_t lds = p.ld_src;
  const C* cscale = static_cast<const C*>(p.colscale);
  const C csa = static_cast<C>(p.cs_a), csb = static_cast<C>(p.cs_b);
  bool own[NV];
#pragma unroll
  for (int m = 0; m < NV; ++m) own[m] = (gl + G * m) < nchunks;

  for (int64_t base = beg; base < end; base += step) {
    const int cnt = static_cast<int>((end - base) < G ? (end - base) : G);
    int myj = 0;
    C myg = C(0);
    if (gl < cnt) {
      myj = stream_load(p.indices + base + gl);
      myg = p.values ? static_cast<C>(stream_load(p.values + base + gl)) : C(1);
      if (cscale) myg *= csa * cscale[myj] + csb;
    }
    int e = 0;
    for (; e + U <= cnt; e += U) {
      int j[U];
      C g[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        j[u] = bcast_i<G>(myj, gbase + e + u);
        g[u] = bcast_f<G>(myg, gbase + e + u);
      }
      // every gather of the batch is issued before the first is consumed; the
      // data stays in its storage form (one 16-byte chunk) until its FMAs
      typename CK::Raw x[U][NV];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int m = 0; m < NV; ++m)
          if (own[m]) x[u][m] = CK::load_raw(src + static_cast<int64_t>(j[u]) * lds + (gl + G * m) * EPC);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int m = 0; m < NV; ++m)
          if (own[m]) {
            C v[EPC];
            CK::unpack(x[u][m], v);
#pragma unroll
            for (int t = 0; t < EPC; ++t) acc[m][t] += g[u] * v[t];
          }
    }
    for (; e < cnt; ++e) {
      const int j = bcast_i<G>(myj, gbase + e);
      const C g = bcast_f<G>(myg, gbase + e);
#pragma unroll
      for (int m = 0; m < NV; ++m) {
        if (own[m]) {
          C x[EPC];
          CK::load(src + static_cast<int64_t>(j) * lds + (gl + G * m) * EPC, x);
#pragma unroll
          for (int t = 0; t < EPC; ++t) acc[m][t] += g * x[t];
        }
      }
    }
  }
}

template <typename T, typename C, int NV, bool VEC>
__device__ inline void epilogue(const SpmmPass& p, int64_t row, int gl, int G, int nchunks,
                                const C (&acc)[NV][Chunk<T, C, VEC>::N]) {
  using CK = Chunk<T, C, VEC>;
  constexpr int EPC = CK::N;
  const C r = p.rowscale ? static_cast<const C*>(p.rowscale)[row] : C(0);
  const C ka = static_cast<C>(p.a0) + static_cast<C>(p.a1) * r;
  const C kb = static_cast<C>(p.b0) + static_cast<C>(p.b1) * r;
  const C kc = static_cast<C>(p.c0) + static_cast<C>(p.c1) * r;
  const C ke = static_cast<C>(p.e);
  const T* add = static_cast<const T*>(p.add);
  T* out = static_cast<T*>(p.out);
  T* out2 = static_cast<T*>(p.out2);
#pragma unroll
  for (int m = 0; m < NV; ++m) {
    const int ch = gl + G * m;
    if (ch >= nchunks) continue;
    const int col0 = ch * EPC;
    const int valid = (p.ncols - col0) < EPC ? (p.ncols - col0) : EPC;
    C y[EPC];
#pragma unroll
    for (int t = 0; t < EPC; ++t) y[t] = ka * acc[m][t];
    if (add) {
      C a[EPC];
      CK::load_stream(add + row * p.ld_add + col0, a);
#pragma unroll
      for (int t = 0; t < EPC; ++t) y[t] += kb * a[t];
    }
    if (p.svec) {
#pragma unroll
      for (int t = 0; t < EPC; ++t)
        if (t < valid) y[t] += ke * static_cast<C>(p.svec[col0 + t]);
    }
    CK::store(out + row * p.ld_out + col0, y, valid);
    if (out2) {
      C z[EPC];
#pragma unroll
      for (int t = 0; t < EPC; ++t) z[t] = kc * acc[m][t];
      CK::store(out2 + row * p.ld_out2 + col0, z, valid);
    }
  }
}

template <typename T, typename C, int G, int NV, bool VEC>
__global__ __launch_bounds__(kThreads) void spmm_pass_kernel(SpmmPass p) {
  using CK = Chunk<T, C, VEC>;
  constexpr int EPC = CK::N;
  __shared__ C red[kWaves][NV * EPC][64];
  const int nchunks = (p.ncols + EPC - 1) / EPC;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  C acc[NV][EPC];
#pragma unroll
  for (int m = 0; m < NV; ++m)
#pragma unroll
    for (int t = 0; t < EPC; ++t) acc[m][t] = C(0);

  if (static_cast<int64_t>(blockIdx.x) < p.n_heavy) {
    // A hub row: the whole block.  Lanes own chunks lane + 64 m (NV covers
    // nchunks for any G because G < 64 implies nchunks <= 32 and NV == 1).
    const int64_t row = p.heavy_rows[blockIdx.x];
    const int64_t beg = p.indptr[row], end = p.indptr[row + 1];
    accumulate<T, C, 64, NV, VEC>(p, beg + 64 * wave, end, 64 * kWaves, lane, 0, nchunks, acc);
#pragma unroll
    for (int m = 0; m < NV; ++m)
#pragma unroll
      for (int t = 0; t < EPC; ++t) red[wave][m * EPC + t][lane] = acc[m][t];
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int m = 0; m < NV; ++m)
#pragma unroll
        for (int t = 0; t < EPC; ++t) {
          C s = red[0][m * EPC + t][lane];
          for (int w = 1; w < kWaves; ++w) s += red[w][m * EPC + t][lane];
          acc[m][t] = s;
        }
      epilogue<T, C, NV, VEC>(p, row, lane, 64, nchunks, acc);
    }
    return;
  }

  constexpr int kRowsPerWave = 64 / G;
  const int64_t lb = static_cast<int64_t>(blockIdx.x) - p.n_heavy;
  const int64_t row = (lb * kWaves + wave) * kRowsPerWave + lane / G;
  if (row >= p.n_rows) return;
  const int64_t beg = p.indptr[row], end = p.indptr[row + 1];
  if (p.heavy_threshold > 0 && end - beg > p.heavy_threshold) return;
  const int gl = lane % G;
  const int gbase = lane - gl;
  accumulate<T, C, G, NV, VEC>(p, beg, end, G, gl, gbase, nchunks, acc);
  epilogue<T, C, NV, VEC>(p, row, gl, G, nchunks, acc);
}

template <typename T, typename C, int G, int NV, bool VEC>
void launch_cfg(const SpmmPass& p, hipStream_t stream) {
  constexpr int kRowsPerBlock = kWaves * (64 / G);
  const int64_t light_blocks = ceil_div(p.n_rows, kRowsPerBlock);
  const int64_t grid = p.n_heavy + light_blocks;
  if (grid == 0) return;
  hipLaunchKernelGGL((spmm_pass_kernel<T, C, G, NV, VEC>), dim3(static_cast<unsigned>(grid)),
                     dim3(kThreads), 0, stream, p);
  ISVD_LAUNCH_CHECK();
}

template <typename T, typename C, bool VEC>
void launch_vec(const SpmmPass& p, hipStream_t stream) {
  constexpr int EPC = Chunk<T, C, VEC>::N;
  const int nchunks = static_cast<int>(ceil_div(p.ncols, EPC));
  if (nchunks <= 8) return launch_cfg<T, C, 8, 1, VEC>(p, stream);
  if (nchunks <= 16) return launch_cfg<T, C, 16, 1, VEC>(p, stream);
  if (nchunks <= 32) return launch_cfg<T, C, 32, 1, VEC>(p, stream);
  if (nchunks <= 64) return launch_cfg<T, C, 64, 1, VEC>(p, stream);
  if (nchunks <= 128) return launch_cfg<T, C, 64, 2, VEC>(p, stream);
  if (nchunks <= 192) return launch_cfg<T, C, 64, 3, VEC>(p, stream);
  if (nchunks <= 256) return launch_cfg<T, C, 64, 4, VEC>(p, stream);
  if (nchunks <= 512) return launch_cfg<T, C, 64, 8, VEC>(p, stream);
  if (nchunks <= 1024) return launch_cfg<T, C, 64, 16, VEC>(p, stream);
  throw Error{ISVD_E_INVALID, "spmm pass: more than 1024 columns"};
}

bool aligned16(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 15u) == 0; }

}  // namespace

template <typename T>
void launch_spmm_pass(const SpmmPass& p, hipStream_t stream) {
  using C = typename ComputeOf<T>::type;
  constexpr int EPC = 16 / sizeof(T);
  ISVD_CHECK(p.ncols >= 1 && p.ncols <= 1024, ISVD_E_INVALID, "spmm pass: ncols out of range");
  // 16-byte chunks only when every row of every block is whole chunks (no read past a row's end)
  bool vec = p.ncols % EPC == 0 && aligned16(p.src) && aligned16(p.out) && p.ld_src % EPC == 0 &&
             p.ld_out % EPC == 0;
  if (p.add) vec = vec && aligned16(p.add) && p.ld_add % EPC == 0;
  if (p.out2) vec = vec && aligned16(p.out2) && p.ld_out2 % EPC == 0;
  void* tok = nullptr;
  if (spmm_profiling()) {
    // Algorithmic bytes of the pass: CSR arrays, gathered rows (every gather
    // counted: "gather-inclusive"; each source row once: "compulsory"), the
    // row-wise streams read and written.
    const double n = static_cast<double>(p.n_rows), l = p.ncols, s = sizeof(T), cs = sizeof(C);
    const double e = static_cast<double>(p.nnz);
    double rows = n * l * s;                                   // out
    if (p.add) rows += n * l * s;
    if (p.out2) rows += n * l * s;
    if (p.rowscale) rows += n * cs;
    double csr = 8.0 * (n + 1) + 4.0 * e + (p.values ? 4.0 * e : 0.0);
    const double gather = csr + rows + e * l * s + (p.colscale ? e * cs : 0.0);
    const double compulsory = csr + rows + n * l * s + (p.colscale ? n * cs : 0.0);
    tok = spmm_profile_begin(stream, gather, compulsory, static_cast<int>(sizeof(T)));
  }
  if (vec) launch_vec<T, C, true>(p, stream);
  else launch_vec<T, C, false>(p, stream);
  if (tok) spmm_profile_end(stream, tok);
}

template void launch_spmm_pass<double>(const SpmmPass&, hipStream_t);
template void launch_spmm_pass<float>(const SpmmPass&, hipStream_t);
template void launch_spmm_pass<bf16>(const SpmmPass&, hipStream_t);

// ---------------------------------------------------------------- column sums

namespace {

constexpr int kColsumMaxPerLane = 16;   // up to 1024 columns

// Each wave streams whole rows (lane j owns columns j, j+64, ...) and keeps
// FP64 sums in registers; waves of a block combine through LDS in order.
template <typename T>
__global__ __launch_bounds__(256) void colsum_partial_kernel(int64_t rows, int cols, const T* y,
                                                             int64_t ld, double* partial) {
  __shared__ double red[4][1024];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int per_lane = (cols + 63) / 64;
  double acc[kColsumMaxPerLane];
#pragma unroll
  for (int m = 0; m < kColsumMaxPerLane; ++m) acc[m] = 0.0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 4;
  int64_t r = static_cast<int64_t>(blockIdx.x) * 4 + wave;
  // four rows in flight per wave
  for (; r + 3 * stride < rows; r += 4 * stride) {
    double x[4][kColsumMaxPerLane];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T* row = y + (r + u * stride) * ld;
#pragma unroll
      for (int m = 0; m < kColsumMaxPerLane; ++m) {
        const int c = lane + 64 * m;
        x[u][m] = (m < per_lane && c < cols) ? static_cast<double>(Elem<T>::load(row + c)) : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int m = 0; m < kColsumMaxPerLane; ++m) acc[m] += x[u][m];
  }
  for (; r < rows; r += stride) {
    const T* row = y + r * ld;
#pragma unroll
    for (int m = 0; m < kColsumMaxPerLane; ++m) {
      const int c = lane + 64 * m;
      if (m < per_lane && c < cols) acc[m] += static_cast<double>(Elem<T>::load(row + c));
    }
  }
#pragma unroll
  for (int m = 0; m < kColsumMaxPerLane; ++m) {
    const int c = lane + 64 * m;
    if (m < per_lane && c < cols) red[wave][c] = acc[m];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < cols; c += blockDim.x)
    partial[static_cast<int64_t>(blockIdx.x) * cols + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
}

// s[c] = sum over parts: one block per column, strided partial sums, fixed-order tree.
__global__ __launch_bounds__(256) void colsum_final_kernel(int nparts, int cols, const double* partial, double* s) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double acc = 0.0;
  for (int q = threadIdx.x; q < nparts; q += 256) acc += partial[static_cast<int64_t>(q) * cols + c];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) s[c] = red[0];
}

}  // namespace

template <typename T>
void launch_colsum(int64_t rows, int cols, const T* y, int64_t ld, double* partial, double* s,
                   hipStream_t stream) {
  ISVD_CHECK(cols >= 1 && cols <= 1024, ISVD_E_INVALID, "colsum: cols out of range");
  const int64_t want = ceil_div(rows > 0 ? rows : 1, 16);
  const int nparts = static_cast<int>(want < kColsumBlocks ? want : kColsumBlocks);
  hipLaunchKernelGGL(colsum_partial_kernel<T>, dim3(nparts), dim3(256), 0, stream, rows, cols, y, ld, partial);
  ISVD_LAUNCH_CHECK();
  hipLaunchKernelGGL(colsum_final_kernel, dim3(cols), dim3(256), 0, stream, nparts, cols, partial, s);
  ISVD_LAUNCH_CHECK();
}

template void launch_colsum<double>(int64_t, int, const double*, int64_t, double*, double*, hipStream_t);
template void launch_colsum<float>(int64_t, int, const float*, int64_t, double*, double*, hipStream_t);
template void launch_colsum<bf16>(int64_t, int, const bf16*, int64_t, double*, double*, hipStream_t);

}  // namespace isvd
