// Dense kernels: FP64-MFMA Gram, MFMA tall GEMM, blocked Cholesky, tall
// triangular solve, one-sided Jacobi SVD, Philox Gaussian block.
//
// MFMA operand layout used throughout (16x16x4, FP32 and FP64): for lane t,
// the A operand is A[t % 16][t / 16] and the B operand is B[t / 16][t % 16].
// Accumulator value r (0..3) of lane t is D[row][t % 16] with
// row = 4 (t / 16) + r for FP32 and row = t / 16 + 4 r for FP64 (drow below;
// measured on gfx950).
#include "dense.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

namespace isvd {

namespace {

__device__ inline v4f mfma4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline v4d mfma4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename C> __device__ inline int drow(int lk, int r);
template <> __device__ inline int drow<float>(int lk, int r) { return 4 * lk + r; }
template <> __device__ inline int drow<double>(int lk, int r) { return lk + 4 * r; }

template <typename C> struct Acc4;
template <> struct Acc4<float> { using type = v4f; };
template <> struct Acc4<double> { using type = v4d; };

template <typename C, typename T>
__device__ inline C ld_as(const T* p) { return static_cast<C>(Elem<T>::load(p)); }

// ============================================================ Gram
//
// C = A^T B over a tall row range with exact products and FP64 sums (FP64
// MFMA 16x16x4).  The 16 x 16 output tiles are grouped in 3 x 3 blocks; each
// wave owns one block ("job") and keeps its nine accumulators in registers,
// so one k-step reads three A and three B fragments for up to nine MFMAs.
// For A^T A only blocks on or above the diagonal exist and tiles below the
// diagonal inside a diagonal block are skipped.  A workgroup holds up to 16
// waves (jobs; for A^T A a whole number of waves per SIMD, jobs placed on the
// SIMDs by cost) and streams one row slice through two LDS buffers (rows staged
// as FP32 for FP32/BF16 inputs, FP64 otherwise): the next chunk is loaded
// into registers while the MFMAs of the current one run, one barrier per
// chunk.  Row slices write partial tiles that a second kernel adds in a
// fixed order.

constexpr int kGramRB = 3;          // tiles per job side
constexpr int kGramMaxWaves = 16;
constexpr int kGramPF = 16;         // staged elements per thread per chunk
constexpr int kGramMaxParts = 256;
constexpr int kGramMinStageWaves = 8;
constexpr size_t kGramMaxLds = 96 * 1024;
constexpr int kGramTableSlots = 64;   // wave slots (groups x waves) a job table can describe

// Job of each wave slot (group * waves + wave) when the plan balances the
// work of A^T A over the SIMDs (0xff: no job); passed by value.
struct GramJobTable {
  uint8_t bi[kGramTableSlots];
  uint8_t bj[kGramTableSlots];
};

template <typename TA, typename TB>
struct GramStage {
  using type = typename std::conditional<std::is_same<TA, double>::value || std::is_same<TB, double>::value,
                                         double, float>::type;
};

// LDS row stride (elements) for `cols` staged columns: consecutive rows start
// 64 bytes apart modulo 256, so the four k-rows of one fragment read fall in
// different banks.
__host__ __device__ inline int gram_lds_ld(int cols, int esize) {
  const int bytes = cols * esize;
  const int pad = ((64 - bytes) % 256 + 256) % 256;
  return (bytes + pad) / esize;
}

// The k-steps of one chunk for one job (a 3 x 3 block of tiles; on a
// diagonal block of A^T A the tiles below its diagonal are skipped).  The
// fragments of the next k-step are read while the MFMAs of the current one run.
template <typename S>
__device__ inline void gram_ksteps(const S* As, const S* Bs, int lda_s, int ldb_s, int nk, int ti0, int tj0, int li,
                                   int lk, bool diag, v4d (&acc)[kGramRB][kGramRB]) {
  const S* pa = As + lk * lda_s + ti0 * 16 + li;
  const S* pb = Bs + lk * ldb_s + tj0 * 16 + li;
  S fa[kGramRB], fb[kGramRB];
#pragma unroll
  for (int r = 0; r < kGramRB; ++r) {
    fa[r] = pa[r * 16];
    fb[r] = pb[r * 16];
  }
  for (int kk = 0; kk < nk; ++kk) {
    double a[kGramRB], b[kGramRB];
#pragma unroll
    for (int r = 0; r < kGramRB; ++r) {
      a[r] = static_cast<double>(fa[r]);
      b[r] = static_cast<double>(fb[r]);
    }
    // next k-step (the last iteration re-reads its own rows: in bounds, unused)
    const int step = kk + 1 < nk ? 4 : 0;
    pa += step * lda_s;
    pb += step * ldb_s;
#pragma unroll
    for (int r = 0; r < kGramRB; ++r) {
      fa[r] = pa[r * 16];
      fb[r] = pb[r * 16];
    }
#pragma unroll
    for (int r = 0; r < kGramRB; ++r)
#pragma unroll
      for (int c = 0; c < kGramRB; ++c)
        if (r <= c) acc[r][c] = mfma4(a[r], b[c], acc[r][c]);
    if (!diag) {
#pragma unroll
      for (int r = 1; r < kGramRB; ++r)
#pragma unroll
        for (int c = 0; c < r; ++c) acc[r][c] = mfma4(a[r], b[c], acc[r][c]);
    }
  }
}

// Two adjacent columns of one row in one load (the address is aligned to
// two elements), converted to the staging type.
template <typename T, typename S> struct Pair;
template <typename S> struct Pair<double, S> {
  __device__ static inline void load(const double* p, S& x, S& y) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    x = static_cast<S>(v.x);
    y = static_cast<S>(v.y);
  }
};
template <typename S> struct Pair<float, S> {
  __device__ static inline void load(const float* p, S& x, S& y) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    x = static_cast<S>(v.x);
    y = static_cast<S>(v.y);
  }
};
template <typename S> struct Pair<bf16, S> {
  __device__ static inline void load(const bf16* p, S& x, S& y) {
    const uint32_t v = *reinterpret_cast<const uint32_t*>(p);
    x = static_cast<S>(bf16_to_float(static_cast<uint16_t>(v & 0xffffu)));
    y = static_cast<S>(bf16_to_float(static_cast<uint16_t>(v >> 16)));
  }
};

// Columns c, c + 1 of a row (c even; zeros at and past `cols`).  BF16 rows
// are kept as loaded (the 32-bit word of a pair, or the zero-extended 16-bit
// element, in v[0]) and widened by gram_widen at staging time: widening at
// load time would make each load wait at once instead of under the MFMAs of
// the current chunk.
template <int VW, typename T, typename S>
__device__ inline void gram_load(const T* row, int c, int cols, bool ok, S (&v)[VW]) {
  if constexpr (std::is_same<T, bf16>::value) {
    static_assert(sizeof(S) == 4, "BF16 rows are staged as FP32");
    // paired BF16 rows have an even column count (gram_impl), so c < cols
    // covers both elements of the word
    uint32_t w = 0;
    if constexpr (VW == 2) {
      if (ok && c < cols) w = *reinterpret_cast<const uint32_t*>(row + c);
    } else {
      if (ok && c < cols) w = row[c].bits;
    }
    v[0] = __uint_as_float(w);
    if constexpr (VW == 2) v[1] = S(0);
  } else if constexpr (VW == 1) {
    v[0] = (ok && c < cols) ? static_cast<S>(Elem<T>::load(row + c)) : S(0);
  } else {
    v[0] = S(0);
    v[1] = S(0);
    if (ok && c + 1 < cols) Pair<T, S>::load(row + c, v[0], v[1]);
    else if (ok && c < cols) v[0] = static_cast<S>(Elem<T>::load(row + c));
  }
}

// The staged values of what gram_load left in v (identity except for BF16).
template <int VW, typename T, typename S>
__device__ inline void gram_widen(const S (&v)[VW], S (&out)[VW]) {
  if constexpr (std::is_same<T, bf16>::value) {
    const uint32_t w = __float_as_uint(v[0]);
    out[0] = __uint_as_float(w << 16);
    if constexpr (VW == 2) out[1] = __uint_as_float(w & 0xffff0000u);
  } else {
#pragma unroll
    for (int e = 0; e < VW; ++e) out[e] = v[e];
  }
}

// Rows staged per wave and chunk: J rows of CS steps of 64 VW columns each
// (for A and, if B differs, for B).
template <typename S, int CS, int VW, bool SAME>
constexpr int gram_rows_per_wave() {
  constexpr int words = CS * VW * static_cast<int>(sizeof(S) / 4) * (SAME ? 1 : 2);
  return kGramPF / words > 0 ? kGramPF / words : 1;
}

template <typename TA, typename TB, int CS, int VW, bool SAME, int KSPLIT>
__global__ __launch_bounds__(64 * kGramMaxWaves) void gram_partial_kernel(
    int64_t rows, int m, int p, const TA* A, int64_t lda, const TB* B, int64_t ldb, int tm, int tp, int nbi,
    int nbj, int njobs, int64_t rows_per_block, int rb, int ldsa, int ldsb, double* partial, int mp, int pp,
    int use_table, GramJobTable table) {
  using S = typename GramStage<TA, TB>::type;
  constexpr int J = gram_rows_per_wave<S, CS, VW, SAME>();
  extern __shared__ __align__(16) unsigned char gram_smem[];
  S* buf0 = reinterpret_cast<S*>(gram_smem);
  const int per_buf = rb * (ldsa + (SAME ? 0 : ldsb));
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int nw = static_cast<int>(blockDim.x >> 6);
  const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  // KSPLIT == 2: waves wv and wv + nj share job wv, each taking half the k-steps
  const int nj = nw / KSPLIT, set = KSPLIT == 1 ? 0 : wv / nj;
  const int job = static_cast<int>(blockIdx.y) * nj + (wv - set * nj);
  bool has_job = job < njobs;
  // job -> block (bi, bj): from the plan's table, else the upper triangle row
  // by row for A^T A and row-major otherwise
  int bi = 0, bj = 0;
  if (use_table) {
    has_job = table.bi[job] != 0xff;
    bi = has_job ? table.bi[job] : 0;
    bj = has_job ? table.bj[job] : 0;
  } else if (has_job) {
    if (SAME) {
      int rest = job;
      while (rest >= nbj - bi) {
        rest -= nbj - bi;
        ++bi;
      }
      bj = bi + rest;
    } else {
      bi = job / nbj;
      bj = job - bi * nbj;
    }
  }
  const int ti0 = kGramRB * bi, tj0 = kGramRB * bj;
  const int mpa = 16 * kGramRB * nbi, ppa = 16 * kGramRB * nbj;   // staged columns: whole blocks
  // Staged columns run to whole blocks (zeros past m and p), so edge blocks
  // are full blocks whose outer tiles are not stored.
  const bool diag = SAME && bi == bj;
  v4d acc[kGramRB][kGramRB];
#pragma unroll
  for (int r = 0; r < kGramRB; ++r)
#pragma unroll
    for (int c = 0; c < kGramRB; ++c) acc[r][c] = v4d{0.0, 0.0, 0.0, 0.0};

  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < rows ? r0 + rows_per_block : rows;
  // wave wv stages chunk rows wv, wv + nw, ...; lane owns columns
  // VW lane + 64 VW s .. + VW - 1
  S pa[J][CS][VW];
  S pb[SAME ? 1 : J][SAME ? 1 : CS][VW];
  auto fetch = [&](int64_t base) {
    const TA* a0 = A + (base + wv) * lda;
    const TB* b0 = B + (base + wv) * ldb;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int rl = wv + nw * j;
      const bool ok = rl < rb && base + rl < r1;   // wave-uniform
      const TA* aj = a0 + static_cast<int64_t>(nw * j) * lda;
#pragma unroll
      for (int s = 0; s < CS; ++s) gram_load<VW>(aj, VW * lane + 64 * VW * s, m, ok, pa[j][s]);
      if constexpr (!SAME) {
        const TB* bj_ = b0 + static_cast<int64_t>(nw * j) * ldb;
#pragma unroll
        for (int s = 0; s < CS; ++s) gram_load<VW>(bj_, VW * lane + 64 * VW * s, p, ok, pb[j][s]);
      }
    }
  };
  auto stage = [&](S* dst) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int rl = wv + nw * j;
      if (rl >= rb) continue;
      S* da = dst + rl * ldsa + VW * lane;
#pragma unroll
      for (int s = 0; s < CS; ++s)
        if (VW * lane + 64 * VW * s < mpa) {
          S w[VW];
          gram_widen<VW, TA, S>(pa[j][s], w);
#pragma unroll
          for (int e = 0; e < VW; ++e) da[64 * VW * s + e] = w[e];
        }
      if constexpr (!SAME) {
        S* db = dst + rb * ldsa + rl * ldsb + VW * lane;
#pragma unroll
        for (int s = 0; s < CS; ++s)
          if (VW * lane + 64 * VW * s < ppa) {
            S w[VW];
            gram_widen<VW, TB, S>(pb[j][s], w);
#pragma unroll
            for (int e = 0; e < VW; ++e) db[64 * VW * s + e] = w[e];
          }
      }
    }
  };
  if (r0 < r1) {
    fetch(r0);
    stage(buf0);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t base = r0; base < r1; base += rb) {
    const bool more = base + rb < r1;
    if (more) fetch(base + rb);
    const S* As = buf0 + cur * per_buf;
    const S* Bs = SAME ? As : As + rb * ldsa;
    const int ldb_s = SAME ? ldsa : ldsb;
    const int nks = rb / (4 * KSPLIT);   // k-steps of this wave in the chunk
    if (has_job)
      gram_ksteps(As + set * nks * 4 * ldsa, Bs + set * nks * 4 * ldb_s, ldsa, ldb_s, nks, ti0, tj0, li, lk, diag,
                  acc);
    if (more) stage(buf0 + (cur ^ 1) * per_buf);
    __syncthreads();
    cur ^= 1;
  }
  if constexpr (KSPLIT == 2) {
    // the staging buffers are free (the chunk loop ends with a barrier)
    double* xch = reinterpret_cast<double*>(gram_smem) + static_cast<int64_t>(wv - set * nj) * kGramRB * kGramRB * 4 * 64;
    if (set == 1 && has_job) {
#pragma unroll
      for (int r = 0; r < kGramRB; ++r)
#pragma unroll
        for (int c = 0; c < kGramRB; ++c)
#pragma unroll
          for (int q = 0; q < 4; ++q) xch[((r * kGramRB + c) * 4 + q) * 64 + lane] = acc[r][c][q];
    }
    __syncthreads();
    if (set == 1) return;
    if (has_job) {
#pragma unroll
      for (int r = 0; r < kGramRB; ++r)
#pragma unroll
        for (int c = 0; c < kGramRB; ++c) {
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[r][c][q] += xch[((r * kGramRB + c) * 4 + q) * 64 + lane];
          __builtin_amdgcn_sched_barrier(0);  // one tile's loads at a time (register budget)
        }
    }
  }
  if (!has_job) return;
  double* part = partial + static_cast<int64_t>(blockIdx.x) * mp * pp;
#pragma unroll
  for (int r = 0; r < kGramRB; ++r)
#pragma unroll
    for (int c = 0; c < kGramRB; ++c) {
      const int ti = ti0 + r, tj = tj0 + c;
      if (ti >= tm || tj >= tp || (SAME && ti > tj)) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        part[static_cast<int64_t>(ti * 16 + drow<double>(lk, q)) * pp + tj * 16 + li] = acc[r][c][q];
    }
}

// C[a][b] = sum over row slices of the partial Gram tiles: 64 outputs per
// block, four interleaved partial sums per output, combined in a fixed order.
// For A^T A only entries a <= b are summed (the partial tiles are exactly
// symmetric) and written to both (a, b) and (b, a).
__global__ __launch_bounds__(256) void gram_reduce_kernel(int m, int p, int nparts, const double* partial, int mp,
                                                          int pp, int same, double* C, int64_t ldc) {
  __shared__ double red[4][64];
  const int e = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 64 + e;
  const bool in = idx < static_cast<int64_t>(m) * p;
  const int a = in ? static_cast<int>(idx / p) : 0, b = in ? static_cast<int>(idx % p) : 0;
  const bool ok = in && (!same || a <= b);
  const int64_t stride = static_cast<int64_t>(mp) * pp;
  const double* src = partial + static_cast<int64_t>(a) * pp + b;
  // four independent sums so that several partial loads are in flight
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (ok) {
    int q = w;
#pragma unroll 2
    for (; q + 12 < nparts; q += 16) {
      s0 += src[q * stride];
      s1 += src[(q + 4) * stride];
      s2 += src[(q + 8) * stride];
      s3 += src[(q + 12) * stride];
    }
    for (; q < nparts; q += 4) s0 += src[q * stride];
  }
  red[w][e] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (w == 0 && ok) {
    const double v = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
    C[static_cast<int64_t>(a) * ldc + b] = v;
    if (same && a != b) C[static_cast<int64_t>(b) * ldc + a] = v;
  }
}

struct GramPlan {
  int mp, pp, tm, tp, nbi, nbj, njobs, waves, groups, vw, cs, rb, ldsa, ldsb, nparts, ksplit;
  int64_t rows_per_block;
  size_t lds;
  bool use_table = false;
  GramJobTable table{};
};

// Balanced placement of the jobs of A^T A.  Waves w, w + 4, w + 8, ... of a
// workgroup share one SIMD, and a workgroup takes as long as its busiest
// SIMD; diagonal blocks cost kGramRB (kGramRB + 1) / 2 MFMAs per k-step,
// the others kGramRB^2.  The plan chooses how many jobs of each kind every
// group holds and spreads them over the group's four SIMDs so that the sum
// over groups of the busiest SIMD's cost is least (exhaustive over the two
// job kinds; every group has `waves` slots, a multiple of four).
void balance_gram_jobs(GramPlan& g) {
  const int nb = g.nbi, k = g.waves / 4, G = g.groups;
  const int cd = kGramRB * (kGramRB + 1) / 2, co = kGramRB * kGramRB;
  const int nd = nb, no = g.njobs - nb;
  // best split of (o, d) jobs over four bins of k slots: least maximum bin cost
  auto bins = [&](int o, int d, int (&bo)[4], int (&bd)[4]) {
    int best = -1;
    for (int o0 = 0; o0 <= std::min(o, k); ++o0)
      for (int o1 = 0; o1 <= std::min(o - o0, k); ++o1)
        for (int o2 = 0; o2 <= std::min(o - o0 - o1, k); ++o2) {
          const int o3 = o - o0 - o1 - o2;
          if (o3 > k) continue;
          int oo[4] = {o0, o1, o2, o3}, dd[4] = {0, 0, 0, 0};
          bool ok = true;
          for (int x = 0; x < d; ++x) {   // each diagonal job to the cheapest bin with room
            int tgt = -1;
            for (int b = 0; b < 4; ++b)
              if (oo[b] + dd[b] < k && (tgt < 0 || co * oo[b] + cd * dd[b] < co * oo[tgt] + cd * dd[tgt])) tgt = b;
            if (tgt < 0) {
              ok = false;
              break;
            }
            ++dd[tgt];
          }
          if (!ok) continue;
          int mx = 0;
          for (int b = 0; b < 4; ++b) mx = std::max(mx, co * oo[b] + cd * dd[b]);
          if (best < 0 || mx < best) {
            best = mx;
            for (int b = 0; b < 4; ++b) {
              bo[b] = oo[b];
              bd[b] = dd[b];
            }
          }
        }
    return best;
  };
  // cost[g][o][d]: least sum of busiest-SIMD costs for groups g.. holding o and d jobs
  const int INF = 1 << 30;
  std::vector<int> cost((G + 1) * (no + 1) * (nd + 1), INF), pick_o(cost.size(), 0), pick_d(cost.size(), 0);
  auto at = [&](int gg, int o, int d) { return (gg * (no + 1) + o) * (nd + 1) + d; };
  cost[at(G, 0, 0)] = 0;
  for (int gg = G - 1; gg >= 0; --gg)
    for (int o = 0; o <= no; ++o)
      for (int d = 0; d <= nd; ++d)
        for (int og = 0; og <= std::min(o, 4 * k); ++og)
          for (int dg = 0; dg <= std::min(d, 4 * k - og); ++dg) {
            const int rest = cost[at(gg + 1, o - og, d - dg)];
            if (rest >= INF) continue;
            int bo[4], bd[4];
            const int c = bins(og, dg, bo, bd);
            if (c < 0 || c + rest >= cost[at(gg, o, d)]) continue;
            cost[at(gg, o, d)] = c + rest;
            pick_o[at(gg, o, d)] = og;
            pick_d[at(gg, o, d)] = dg;
          }
  if (cost[at(0, no, nd)] >= INF) return;
  // job lists in the row-by-row order of the upper triangle
  std::vector<std::pair<int, int>> diag, off;
  for (int bi = 0; bi < nb; ++bi)
    for (int bj = bi; bj < nb; ++bj) (bi == bj ? diag : off).push_back({bi, bj});
  for (int e = 0; e < kGramTableSlots; ++e) g.table.bi[e] = g.table.bj[e] = 0xff;
  size_t io = 0, id = 0;
  int o = no, d = nd;
  for (int gg = 0; gg < G; ++gg) {
    const int og = pick_o[at(gg, o, d)], dg = pick_d[at(gg, o, d)];
    int bo[4], bd[4];
    bins(og, dg, bo, bd);
    for (int b = 0; b < 4; ++b) {
      int slot = 0;
      for (int x = 0; x < bo[b]; ++x, ++slot) {
        const int e = gg * g.waves + b + 4 * slot;
        g.table.bi[e] = static_cast<uint8_t>(off[io].first);
        g.table.bj[e] = static_cast<uint8_t>(off[io++].second);
      }
      for (int x = 0; x < bd[b]; ++x, ++slot) {
        const int e = gg * g.waves + b + 4 * slot;
        g.table.bi[e] = static_cast<uint8_t>(diag[id].first);
        g.table.bj[e] = static_cast<uint8_t>(diag[id++].second);
      }
    }
    o -= og;
    d -= dg;
  }
  g.use_table = true;
}

// Row slices: at most kGramMaxParts (one per CU), each a multiple of 16 rows
// (at least 64), so that large blocks use every CU.
int64_t gram_rows_per_part(int64_t rows, int max_parts = kGramMaxParts) {
  const int64_t want = ceil_div(rows > 0 ? rows : 1, max_parts);
  return round_up(want < 64 ? 64 : want, 16);
}

constexpr int kGramCS2[] = {1, 2, 3, 4, 5, 6, 8, 16};   // paired-column loads
constexpr int kGramCS1[] = {1, 2, 4, 8, 16, 32};          // one column per load

GramPlan plan_gram(int64_t rows, int m, int p, bool same, int esize, bool paired, int max_parts) {
  GramPlan g;
  g.mp = pad16(m);
  g.pp = pad16(p);
  g.tm = g.mp / 16;
  g.tp = g.pp / 16;
  g.nbi = static_cast<int>(ceil_div(g.tm, kGramRB));
  g.nbj = static_cast<int>(ceil_div(g.tp, kGramRB));
  g.njobs = same ? g.nbi * (g.nbi + 1) / 2 : g.nbi * g.nbj;
  g.groups = static_cast<int>(ceil_div(g.njobs, kGramMaxWaves));
  g.waves = static_cast<int>(ceil_div(g.njobs, g.groups));
  const int mpa = 16 * kGramRB * g.nbi, ppa = 16 * kGramRB * g.nbj;   // staged columns: whole blocks
  g.vw = paired ? 2 : 1;
  const int need = static_cast<int>(ceil_div(same ? mpa : std::max(mpa, ppa), 64 * g.vw));
  g.cs = 0;
  if (paired) {
    for (int c : kGramCS2)
      if (c >= need) {
        g.cs = c;
        break;
      }
  } else {
    for (int c : kGramCS1)
      if (c >= need) {
        g.cs = c;
        break;
      }
  }
  ISVD_CHECK(g.cs > 0, ISVD_E_INVALID, "gram: more than 2048 columns");
  // One wave per job leaves the four SIMDs of a CU unevenly loaded when the
  // job count is not a multiple of four (A^T A with l = 144: six jobs, two
  // SIMDs with two jobs each); then two waves share each job, taking the two
  // halves of every chunk's k-steps, and their sums meet in LDS at the end.
  g.ksplit = (same && g.cs <= 4 && g.groups == 1 && g.njobs % 4 != 0 && 2 * g.njobs <= kGramMaxWaves) ? 2 : 1;
  g.waves *= g.ksplit;
  // A^T A with one wave per job: whole SIMD rows of waves, jobs placed by cost
  // (the placement depends only on the block count and the group shape, so it
  // is worked out once per shape)
  if (same && g.ksplit == 1) {
    const int w4 = static_cast<int>(round_up(ceil_div(g.njobs, g.groups), 4));
    if (g.groups * w4 <= kGramTableSlots) {
      g.waves = w4;
      static std::mutex mu;
      static std::map<std::tuple<int, int, int>, std::pair<bool, GramJobTable>> placed;
      std::lock_guard<std::mutex> lk(mu);
      const auto key = std::make_tuple(g.nbi, g.waves, g.groups);
      auto it = placed.find(key);
      if (it == placed.end()) {
        balance_gram_jobs(g);
        it = placed.emplace(key, std::make_pair(g.use_table, g.table)).first;
      }
      g.use_table = it->second.first;
      g.table = it->second.second;
    }
  }
  // A^T B with few jobs (a narrow B): waves without a job still stage rows,
  // so that each chunk is deep enough to hide the load latency
  if (!same && g.groups == 1 && g.waves < kGramMinStageWaves) g.waves = kGramMinStageWaves;
  const int words = g.cs * g.vw * esize / 4 * (same ? 1 : 2);
  const int J = kGramPF / words > 0 ? kGramPF / words : 1;
  if (g.waves * J < 4) g.waves = static_cast<int>(ceil_div(4, J));   // at least one k-step per chunk
  g.ldsa = gram_lds_ld(mpa, esize);
  g.ldsb = same ? 0 : gram_lds_ld(ppa, esize);
  const int rstep = 4 * g.ksplit;   // whole k-steps for every wave sharing a job
  if (g.waves * J < rstep) g.waves = static_cast<int>(ceil_div(rstep, J));
  g.rb = (g.waves * J) / rstep * rstep;
  if (g.rb > 64) g.rb = 64;
  while (g.rb > rstep && static_cast<size_t>(2) * g.rb * (g.ldsa + g.ldsb) * esize > kGramMaxLds) g.rb -= rstep;
  ISVD_CHECK(static_cast<size_t>(2) * g.rb * (g.ldsa + g.ldsb) * esize <= kGramMaxLds, ISVD_E_INVALID,
             "gram: block too wide");
  g.lds = static_cast<size_t>(2) * g.rb * (g.ldsa + g.ldsb) * esize;
  // the second wave of each shared job hands its accumulators over in LDS
  if (g.ksplit == 2)
    g.lds = std::max(g.lds, static_cast<size_t>(g.waves / 2) * kGramRB * kGramRB * 4 * 64 * sizeof(double));
  g.rows_per_block = gram_rows_per_part(rows, max_parts);
  g.nparts = static_cast<int>(ceil_div(rows > 0 ? rows : 1, g.rows_per_block));
  return g;
}

template <typename TA, typename TB, int CS, int VW, bool SAME>
void gram_launch(const GramPlan& g, int64_t rows, int m, int p, const TA* A, int64_t lda, const TB* B, int64_t ldb,
                 double* work, hipStream_t stream) {
  // two waves per job only for small A^T A (at most three 3 x 3 blocks a side)
  if constexpr (SAME && CS <= 4) {
    if (g.ksplit == 2) {
      hipLaunchKernelGGL((gram_partial_kernel<TA, TB, CS, VW, SAME, 2>), dim3(g.nparts, g.groups), dim3(64 * g.waves),
                         g.lds, stream, rows, m, p, A, lda, B, ldb, g.tm, g.tp, g.nbi, g.nbj, g.njobs,
                         g.rows_per_block, g.rb, g.ldsa, g.ldsb, work, g.mp, g.pp, 0, g.table);
      ISVD_LAUNCH_CHECK();
      return;
    }
  }
  ISVD_CHECK(g.ksplit == 1, ISVD_E_INVALID, "gram: split jobs need a small A^T A");
  hipLaunchKernelGGL((gram_partial_kernel<TA, TB, CS, VW, SAME, 1>), dim3(g.nparts, g.groups), dim3(64 * g.waves),
                     g.lds, stream, rows, m, p, A, lda, B, ldb, g.tm, g.tp, g.nbi, g.nbj, g.njobs, g.rows_per_block,
                     g.rb, g.ldsa, g.ldsb, work, g.mp, g.pp, g.use_table ? 1 : 0, g.table);
  ISVD_LAUNCH_CHECK();
}

template <typename TA, typename TB, int CS, int VW>
void gram_launch_cs(const GramPlan& g, int64_t rows, int m, int p, const TA* A, int64_t lda, const TB* B,
                    int64_t ldb, bool same, double* work, hipStream_t stream) {
  if constexpr (std::is_same<TA, TB>::value) {
    if (same) return gram_launch<TA, TB, CS, VW, true>(g, rows, m, p, A, lda, B, ldb, work, stream);
  }
  gram_launch<TA, TB, CS, VW, false>(g, rows, m, p, A, lda, B, ldb, work, stream);
}

template <typename T>
bool gram_pair_ok(const T* ptr, int64_t ld) {
  return ld % 2 == 0 && (reinterpret_cast<uintptr_t>(ptr) % (2 * sizeof(T))) == 0;
}

template <typename TA, typename TB>
void gram_impl(int64_t rows, int m, int p, const TA* A, int64_t lda, const TB* B, int64_t ldb,
               bool same, double* C, int64_t ldc, double* work, hipStream_t stream, int max_parts = kGramMaxParts) {
  using S = typename GramStage<TA, TB>::type;
  // BF16 pairs are loaded as one word without a tail case: even column counts only
  const bool even_cols = (!std::is_same<TA, bf16>::value || m % 2 == 0) && (!std::is_same<TB, bf16>::value || p % 2 == 0);
  const bool paired = gram_pair_ok(A, lda) && (same || gram_pair_ok(B, ldb)) && even_cols;
  const GramPlan g = plan_gram(rows, m, p, same, static_cast<int>(sizeof(S)), paired, max_parts);
  if (paired) {
    switch (g.cs) {
      case 1: gram_launch_cs<TA, TB, 1, 2>(g, rows, m, p, A, lda, B, ldb, same, work, stream); break;
      case 2: gram_launch_cs<TA, TB, 2, 2>(g, rows, m, p, A, lda, B, ldb, same, work, stream); break;
      case 3: gram_launch_cs<TA, TB, 3, 2>(g, rows, m, p, A, lda, B, ldb, same, work, stream); break;
      case 4: gram_launch_cs<TA, TB, 4, 2>(g, rows, m, p, A, lda, B, ldb, same, work, stream); break;
      case 5: gram_launch_cs<TA, TB, 5, 2>(g, rows, m, p, A, lda, B, ldb, same, work, stream); break;
      case 6: gram_launch_cs<TA, TB, 6, 2>(g, rows, m, p, A, lda, B, ldb, same, work, stream); break;
      case 8: gram_launch_cs<TA, TB, 8, 2>(g, rows, m, p, A, lda, B, ldb, same, work, stream); break;
      default: gram_launch_cs<TA, TB, 16, 2>(g, rows, m, p, A, lda, B, ldb, same, work, stream); break;
    }
  } else {
    switch (g.cs) {
      case 1: gram_launch_cs<TA, TB, 1, 1>(g, rows, m, p, A, lda, B, ldb, same, work, stream); break;
      case 2: gram_launch_cs<TA, TB, 2, 1>(g, rows, m, p, A, lda, B, ldb, same, work, stream); break;
      case 4: gram_launch_cs<TA, TB, 4, 1>(g, rows, m, p, A, lda, B, ldb, same, work, stream); break;
      case 8: gram_launch_cs<TA, TB, 8, 1>(g, rows, m, p, A, lda, B, ldb, same, work, stream); break;
      case 16: gram_launch_cs<TA, TB, 16, 1>(g, rows, m, p, A, lda, B, ldb, same, work, stream); break;
      default: gram_launch_cs<TA, TB, 32, 1>(g, rows, m, p, A, lda, B, ldb, same, work, stream); break;
    }
  }
  const int64_t total = static_cast<int64_t>(m) * p;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(static_cast<unsigned>(ceil_div(total, 64))), dim3(256),
                     0, stream, m, p, g.nparts, work, g.mp, g.pp, same ? 1 : 0, C, ldc);
  ISVD_LAUNCH_CHECK();
}

// ============================================================ tall GEMM

constexpr int kGemmBK = 16;

template <typename T, typename C, int TN, int EPI>
__global__ __launch_bounds__(256) void gemm_tall_kernel(int64_t M, int N, int K1, const T* A1,
                                                        int64_t lda1, int K2, const T* A2,
                                                        int64_t lda2, const C* B, int64_t ldb, T* Cm,
                                                        int64_t ldc, C alpha, C beta,
                                                        double* colpart, int64_t row_tiles) {
  using V = typename Acc4<C>::type;
  __shared__ C As[64][kGemmBK + 1];
  __shared__ C Bs[kGemmBK][16 * TN];
  __shared__ double red[4][16 * TN];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int col0 = blockIdx.y * 16 * TN;
  const int K = K1 + K2;
  double cn[TN];
#pragma unroll
  for (int t = 0; t < TN; ++t) cn[t] = 0.0;

  for (int64_t bt = blockIdx.x; bt < row_tiles; bt += gridDim.x) {
    const int64_t row0 = bt * 64;
    V acc[TN];
#pragma unroll
    for (int t = 0; t < TN; ++t) acc[t] = V{0, 0, 0, 0};
    for (int k0 = 0; k0 < K; k0 += kGemmBK) {
      __syncthreads();
      for (int f = threadIdx.x; f < 64 * kGemmBK; f += 256) {
        const int r = f / kGemmBK, c = f % kGemmBK;
        const int64_t row = row0 + r;
        const int kc = k0 + c;
        C v = C(0);
        if (row < M && kc < K)
          v = kc < K1 ? ld_as<C>(A1 + row * lda1 + kc) : ld_as<C>(A2 + row * lda2 + (kc - K1));
        As[r][c] = v;
      }
      for (int f = threadIdx.x; f < kGemmBK * 16 * TN; f += 256) {
        const int r = f / (16 * TN), c = f % (16 * TN);
        const int kc = k0 + r, col = col0 + c;
        Bs[r][c] = (kc < K && col < N) ? B[static_cast<int64_t>(kc) * ldb + col] : C(0);
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < kGemmBK / 4; ++kk) {
        const C a = As[wave * 16 + li][kk * 4 + lk];
#pragma unroll
        for (int t = 0; t < TN; ++t) acc[t] = mfma4(a, Bs[kk * 4 + lk][t * 16 + li], acc[t]);
      }
    }
    if constexpr (EPI == static_cast<int>(GemmEpi::Store)) {
#pragma unroll
      for (int t = 0; t < TN; ++t) {
        const int col = col0 + t * 16 + li;
        if (col >= N) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = row0 + wave * 16 + drow<C>(lk, r);
          if (row >= M) continue;
          C v = alpha * acc[t][r];
          if (beta != C(0)) v += beta * ld_as<C>(Cm + row * ldc + col);
          Elem<T>::store(Cm + row * ldc + col, v);
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < TN; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = row0 + wave * 16 + drow<C>(lk, r);
          const double v = static_cast<double>(acc[t][r]);
          if (row < M) cn[t] += v * v;
        }
    }
  }
  if constexpr (EPI == static_cast<int>(GemmEpi::ColNorm2)) {
#pragma unroll
    for (int t = 0; t < TN; ++t) {
      double s = cn[t];
      s += __shfl_xor(s, 16, 64);
      s += __shfl_xor(s, 32, 64);
      if (lk == 0) red[wave][t * 16 + li] = s;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < 16 * TN; c += 256) {
      const int col = col0 + c;
      if (col < N) colpart[static_cast<int64_t>(blockIdx.x) * N + col] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
    }
  }
}

__global__ __launch_bounds__(256) void colpart_reduce_kernel(int nparts, int N, const double* part, double* out) {
  __shared__ double s[256];
  const int col = blockIdx.x;
  double acc = 0.0;
  for (int q = threadIdx.x; q < nparts; q += 256) acc += part[static_cast<int64_t>(q) * N + col];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[col] = s[0];
}

constexpr int kColnormParts = 1024;
constexpr int kTrsmParts = 1024;

// FP32 C = alpha A B for K = 16 KC, KC in {4, 5, 8, 9} (no second A block, beta = 0):
// the column block of B (K x 16 TN) is staged in LDS once per workgroup;
// each wave takes 16-row tiles of A straight from memory into registers
// (lane (li, lk) loads A[li][16 c + 4 lk .. +3] as one 16-byte word, c <
// KC) and multiplies them with MFMA 16x16x4, step (c, e) taking
// k = 16 c + e + 4 lk' over the four k-lanes (the same k order is used for
// B's LDS rows, and the sum over k does not depend on it).  No barrier after
// the B stage.
constexpr int kGrWaves = 8;
constexpr size_t kGrMaxLds = 96 * 1024;

template <int TN, int KC>
__global__ __launch_bounds__(64 * kGrWaves) void gemm_rows_kernel(int64_t M, int N, const float* A,
                                                                  int64_t lda, const float* B, int64_t ldb,
                                                                  float* Cm, int64_t ldc, float alpha,
                                                                  int64_t row_tiles, int ldsb) {
  extern __shared__ __align__(16) float gr_smem[];
  const int K = 16 * KC;
  const int col0 = static_cast<int>(blockIdx.y) * 16 * TN;
  for (int f = threadIdx.x; f < K * 16 * TN; f += blockDim.x) {
    const int r = f / (16 * TN), c = f - r * (16 * TN);
    const int col = col0 + c;
    gr_smem[r * ldsb + c] = col < N ? B[static_cast<int64_t>(r) * ldb + col] : 0.0f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kGrWaves;
  // the next tile's A words are loaded while the current tile's MFMAs run
  auto load_tile = [&](int64_t tile, v4f (&a)[KC]) {
    const int64_t row = tile * 16 + li;
    const bool ok = tile < row_tiles && row < M;
    const float* ap = A + (ok ? row : 0) * lda + 4 * lk;
#pragma unroll
    for (int c = 0; c < KC; ++c) a[c] = ok ? *reinterpret_cast<const v4f*>(ap + 16 * c) : v4f{0.f, 0.f, 0.f, 0.f};
  };
  v4f a0[KC], a1[KC];
  int64_t tile = static_cast<int64_t>(blockIdx.x) * kGrWaves + wave;
  load_tile(tile, a0);
  auto step = [&](int64_t t0, v4f (&cur)[KC], v4f (&nxt)[KC]) {
    load_tile(t0 + stride, nxt);
    v4f acc[TN];
#pragma unroll
    for (int t = 0; t < TN; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < KC; ++c) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float* brow = gr_smem + (16 * c + 4 * lk + e) * ldsb + li;
#pragma unroll
        for (int t = 0; t < TN; ++t) acc[t] = mfma4(cur[c][e], brow[16 * t], acc[t]);
        __builtin_amdgcn_sched_barrier(0);  // one k-step's B operands live at a time
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    float* crow[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) crow[r] = Cm + (t0 * 16 + drow<float>(lk, r)) * ldc + col0 + li;
#pragma unroll
    for (int t = 0; t < TN; ++t) {
      if (col0 + 16 * t + li < N) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (t0 * 16 + drow<float>(lk, r) < M) crow[r][16 * t] = alpha * acc[t][r];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  while (tile < row_tiles) {
    step(tile, a0, a1);
    tile += stride;
    if (tile >= row_tiles) break;
    step(tile, a1, a0);
    tile += stride;
  }
}

// Uses gemm_rows_kernel when the shape and alignment allow; returns false otherwise.
bool gemm_rows_try(int64_t M, int N, int K, const float* A, int64_t lda, const float* B, int64_t ldb, float* Cm,
                   int64_t ldc, double alpha, hipStream_t stream) {
  const int kc = K / 16;
  if (K % 16 != 0 || !(kc == 4 || kc == 5 || kc == 8 || kc == 9) || lda % 4 != 0 ||
      reinterpret_cast<uintptr_t>(A) % 16 != 0)
    return false;
  const int tiles = static_cast<int>(ceil_div(N, 16));
  int tn_max = static_cast<int>((kGrMaxLds / (sizeof(float) * K) - 4) / 16);
  tn_max = std::min(tn_max, 11);
  if (tn_max < 1) return false;
  const int ncb = static_cast<int>(ceil_div(tiles, tn_max));
  const int tn = static_cast<int>(ceil_div(tiles, ncb));
  const int ldsb = 16 * tn + 4;
  const size_t lds = static_cast<size_t>(K) * ldsb * sizeof(float);
  const int64_t row_tiles = ceil_div(M, 16);
  // one workgroup per compute unit and column block (B is staged once per workgroup)
  static const int cus = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 256;
    return n > 0 ? n : 256;
  }();
  const int64_t want = ceil_div(row_tiles, kGrWaves);
  const unsigned gx = static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(want, std::max(1, cus / ncb))));
  const dim3 grid(gx, static_cast<unsigned>(ncb)), block(64 * kGrWaves);
  const float al = static_cast<float>(alpha);
  auto go = [&](auto tn_c, auto kc_c) {
    constexpr int TNv = decltype(tn_c)::value, KCv = decltype(kc_c)::value;
    hipLaunchKernelGGL((gemm_rows_kernel<TNv, KCv>), grid, block, lds, stream, M, N, A, lda, B, ldb, Cm, ldc, al,
                       row_tiles, ldsb);
  };
  auto with_kc = [&](auto tn_c) {
    switch (K / 16) {
      case 4: go(tn_c, std::integral_constant<int, 4>{}); return true;
      case 5: go(tn_c, std::integral_constant<int, 5>{}); return true;
      case 8: go(tn_c, std::integral_constant<int, 8>{}); return true;
      case 9: go(tn_c, std::integral_constant<int, 9>{}); return true;
      default: return false;
    }
  };
  bool launched = false;
  switch (tn) {
#define ISVD_GR(X) \
  case X: launched = with_kc(std::integral_constant<int, X>{}); break;
    ISVD_GR(1) ISVD_GR(2) ISVD_GR(3) ISVD_GR(4) ISVD_GR(5) ISVD_GR(6) ISVD_GR(7) ISVD_GR(8) ISVD_GR(9)
    ISVD_GR(10) ISVD_GR(11)
#undef ISVD_GR
    default: break;
  }
  if (!launched) return false;
  ISVD_LAUNCH_CHECK();
  return true;
}

template <typename T, typename C, int TN>
void gemm_launch_tn(int64_t M, int N, int K1, const T* A1, int64_t lda1, int K2, const T* A2,
                    int64_t lda2, const C* B, int64_t ldb, T* Cm, int64_t ldc, double alpha,
                    double beta, GemmEpi epi, double* colnorm, double* work, hipStream_t stream) {
  const int64_t row_tiles = ceil_div(M, 64);
  const int ycb = static_cast<int>(ceil_div(N, 16 * TN));
  if (epi == GemmEpi::Store) {
    hipLaunchKernelGGL((gemm_tall_kernel<T, C, TN, 0>), dim3(static_cast<unsigned>(row_tiles), ycb),
                       dim3(256), 0, stream, M, N, K1, A1, lda1, K2, A2, lda2, B, ldb, Cm, ldc,
                       static_cast<C>(alpha), static_cast<C>(beta), nullptr, row_tiles);
    ISVD_LAUNCH_CHECK();
  } else {
    const int parts = static_cast<int>(row_tiles < kColnormParts ? row_tiles : kColnormParts);
    hipLaunchKernelGGL((gemm_tall_kernel<T, C, TN, 1>), dim3(parts, ycb), dim3(256), 0, stream, M, N,
                       K1, A1, lda1, K2, A2, lda2, B, ldb, Cm, ldc, static_cast<C>(alpha),
                       static_cast<C>(beta), work, row_tiles);
    ISVD_LAUNCH_CHECK();
    hipLaunchKernelGGL(colpart_reduce_kernel, dim3(N), dim3(256), 0, stream, parts, N, work, colnorm);
    ISVD_LAUNCH_CHECK();
  }
}

// ============================================================ Cholesky

// Orders LDS accesses of one wave: LDS operations of a wave execute in
// program order, so a compiler barrier plus wave-scope fences suffice.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Working storage of the blocked factorisation: the upper tiles (I <= J) of an
// lp x lp matrix, either packed in LDS (small l) or in a global lp x lp array;
// the choice is a template argument so LDS accesses compile to LDS
// instructions (a run-time choice would make every access a generic one).
template <bool kLds>
struct TileStore {
  double* p;  // kLds: packed upper tiles, 256 doubles each; else lp x lp row-major
  int T, lp;
  __device__ inline double& at(int I, int J, int r, int c) const {
    if constexpr (kLds) return p[(I * T - I * (I - 1) / 2 + (J - I)) * 256 + r * 16 + c];
    return p[static_cast<int64_t>(I * 16 + r) * lp + J * 16 + c];
  }
};

constexpr int kCholLdsMaxTiles = 11;   // 66 packed tiles = 132 KB of LDS
constexpr int kJacobiMaxNForChol = 1024;  // l <= 1024

// Value of lane n of each 16-lane row, given to every lane of that row (DPP
// row broadcast, one 64-bit move).  n must fold to a constant.
template <int N>
__device__ inline double row_bcast_n(double v) {
  return __longlong_as_double(__builtin_amdgcn_mov_dpp(__double_as_longlong(v), 0x150 + N, 0xF, 0xF, true));
}
__device__ __forceinline__ double row_bcast(double v, int n) {
  switch (n) {
    case 0: return row_bcast_n<0>(v);
    case 1: return row_bcast_n<1>(v);
    case 2: return row_bcast_n<2>(v);
    case 3: return row_bcast_n<3>(v);
    case 4: return row_bcast_n<4>(v);
    case 5: return row_bcast_n<5>(v);
    case 6: return row_bcast_n<6>(v);
    case 7: return row_bcast_n<7>(v);
    case 8: return row_bcast_n<8>(v);
    case 9: return row_bcast_n<9>(v);
    case 10: return row_bcast_n<10>(v);
    case 11: return row_bcast_n<11>(v);
    case 12: return row_bcast_n<12>(v);
    case 13: return row_bcast_n<13>(v);
    case 14: return row_bcast_n<14>(v);
    default: return row_bcast_n<15>(v);
  }
}

// The same in registers: lane c of each 16-lane row holds column c of the
// tile (the four rows of the wave hold the same columns and compute the same
// values); pivots and row entries reach the other lanes by row broadcasts.
// Row j of the factor is W_j. / r_j; lane a's entry is formed from its
// unscaled value with the same rounding lane a applies, so the update does
// not wait for the scaling.  The column loop touches no memory and takes no
// branch (selects only); lane c keeps its own pivot and checks it at the end.
// X = R^-1 is then solved column by column (lane c: R x = e_c by back
// substitution, each finished x_k folded into the remaining rows).
template <bool kLds>
__device__ __forceinline__ void diag_tile_regs(const TileStore<kLds>& W, int J, double* X, const double* refd,
                                               double rel_tol, int lane, int* bad) {
  const int c = lane & 15;
  double s[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) s[i] = (i <= c) ? W.at(J, J, i, c) : 0.0;
  const double ref_c = refd[J * 16 + c];
  double d_c = 0.0, rinv_c = 0.0;  // lane c: pivot of column c and 1 / R[c][c]
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const double d = row_bcast(s[j], j);
    // 1/sqrt(d) from the hardware estimate and two Newton-Raphson steps
    // (y <- y + y (1 - d y^2) / 2, error squared each step), r = d / sqrt(d)
    const double dd = d > 0.0 ? d : 1e-300;
    double ri = __builtin_amdgcn_rsq(dd);
#pragma unroll
    for (int it = 0; it < 2; ++it) ri = fma(0.5 * ri, fma(-dd * ri, ri, 1.0), ri);
    const double r = dd * ri;
    const double rc = s[j] * ri;  // R[j][c]
    // lanes c < a update s[a] too: entries below the diagonal are never read
    // (broadcasts take s[i] from lanes k > i) and are zeroed on the way out
#pragma unroll
    for (int a = j + 1; a < 16; ++a) {
      const double t = row_bcast(s[j], a) * ri;  // R[j][a]
      s[a] = fma(-t, rc, s[a]);
    }
    s[j] = (c == j) ? r : ((c > j) ? rc : s[j]);
    d_c = (c == j) ? d : d_c;
    rinv_c = (c == j) ? ri : rinv_c;
    __builtin_amdgcn_sched_barrier(0);  // keep the broadcasts of later columns from piling up
  }
  if (lane < 16 && (!(d_c > rel_tol * ref_c) || !isfinite(d_c))) *bad = 1;
  // lane c: s[i] = R[i][c] for i <= c, 0 below.  All four rows store the
  // same values (no branch).
  double acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.0;
#pragma unroll
  for (int k = 15; k >= 0; --k) {
    const double xk = ((k == c ? 1.0 : 0.0) - acc[k]) * row_bcast(rinv_c, k);
    X[k * 16 + c] = xk;
#pragma unroll
    for (int i = 0; i < k; ++i) acc[i] = fma(row_bcast(s[i], k), xk, acc[i]);  // R[i][k] x_k
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) W.at(J, J, i, c) = (i <= c) ? s[i] : 0.0;
  wave_lds_sync();
}

constexpr int kCholThreads = 512;

// retry = 0: factor G + shift I; flag[0] = 1 on breakdown (pivot <= rel_tol x
// its original diagonal, or not finite), else 0.
// retry = 1 (the repair launch queued after every factorisation): nothing
// unless flag[0] is set; then factor G + s I with s = shift x tr(G) and no
// pivot threshold (shifted Cholesky QR), add one to flag[2] and set flag[1]
// if this factorisation breaks down too or tr(G) is not positive and finite.
template <typename C, bool kLds>
__global__ __launch_bounds__(kCholThreads) void cholesky_kernel(int l, const double* G, int64_t ldg, double shift,
                                                        double rel_tol, double* R64, C* Rc, C* Dc, int* flag,
                                                        int retry) {
  extern __shared__ double chol_lds[];
  const int lp = pad16(l), T = lp / 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  __shared__ double X[256];
  __shared__ double refd[kJacobiMaxNForChol];
  __shared__ int bad;
  __shared__ double tr_part[kCholThreads / 64];
  __shared__ double tr_shift;
  __shared__ int skip, tr_bad;
  if (retry) {
    if (tid == 0) skip = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    __syncthreads();
    if (skip) return;
    double part = 0.0;
    for (int i = tid; i < l; i += blockDim.x) part += G[static_cast<int64_t>(i) * ldg + i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    if (lane == 0) tr_part[wave] = part;
    __syncthreads();
    if (tid == 0) {
      double tr = 0.0;
      for (int w = 0; w < nw; ++w) tr += tr_part[w];
      tr_bad = !(tr > 0.0 && isfinite(tr));
      tr_shift = shift * tr;
    }
    __syncthreads();
    shift = tr_shift;
    rel_tol = 0.0;
  }
  const TileStore<kLds> W{kLds ? chol_lds : R64, T, lp};
  for (int i = tid; i < lp; i += blockDim.x)
    refd[i] = i < l ? fabs(G[static_cast<int64_t>(i) * ldg + i] + shift) : 1.0;
  // W = G + shift I on the upper tiles, identity on the padding.  Thread tid
  // takes elements tid, tid + N, ... (row-major, N threads); their (row,
  // column) advance by (N / lp, N % lp) with one carry, so no division per
  // element, and each batch of kLoadU loads is unconditional (clamped
  // addresses) so the whole batch is in flight at once.
  constexpr int kLoadU = 16;
  const int stride_i = kCholThreads / lp, stride_j = kCholThreads - stride_i * lp;
  auto advance = [&](int& i, int& j) {
    i += stride_i;
    j += stride_j;
    if (j >= lp) {
      j -= lp;
      ++i;
    }
  };
  // (A value select would let the compiler move each load into its own
  // branch and wait for it there, so elements outside the matrix load a
  // clamped address and are masked arithmetically: v = g m + a.  Elements
  // with no place in the packed tiles are written to a junk slot.)
  __shared__ double junk;
  {
    int ci = tid / lp, cj = tid - (tid / lp) * lp;
    while (ci < lp) {
      double v[kLoadU];
      int ii[kLoadU], jj[kLoadU];
#pragma unroll
      for (int u = 0; u < kLoadU; ++u) {
        ii[u] = ci;
        jj[u] = cj;
        const bool in = ci < l && cj < l;
        const double gv = G[static_cast<int64_t>(ci < l ? ci : l - 1) * ldg + (cj < l ? cj : l - 1)];
        v[u] = fma(gv, in ? 1.0 : 0.0, ci == cj ? (in ? shift : 1.0) : 0.0);
        advance(ci, cj);
      }
#pragma unroll
      for (int u = 0; u < kLoadU; ++u) {
        const int i = ii[u] < lp ? ii[u] : 0, j = jj[u];
        const bool keep = ii[u] < lp && (i >> 4) <= (j >> 4);
        double* dst = keep ? &W.at(i >> 4, j >> 4, i & 15, j & 15) : &junk;
        *dst = v[u];
      }
    }
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  // one trailing tile: W_KK2 -= R_JK^T R_JK2
  auto trail = [&](int J, int K, int K2) {
    v4d acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = W.at(K, K2, drow<double>(lk, r), li);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int kr = kk * 4 + lk;
      acc = mfma4(-W.at(J, K, kr, li), W.at(J, K2, kr, li), acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) W.at(K, K2, drow<double>(lk, r), li) = acc[r];
  };
  auto factor_diag = [&](int J) {
    diag_tile_regs(W, J, X, refd, rel_tol, lane, &bad);
    for (int e = lane; e < 256; e += 64) Dc[J * 256 + e] = static_cast<C>(X[e]);
  };
  if (wave == 0) factor_diag(0);
  __syncthreads();
  for (int J = 0; J < T; ++J) {
    // panel: R_JK = (R_JJ^-1)^T W_JK for K > J
    for (int K = J + 1 + wave; K < T; K += nw) {
      v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int kr = kk * 4 + lk;
        acc = mfma4(X[kr * 16 + li], W.at(J, K, kr, li), acc);
      }
      // all lanes read their operands before any lane overwrites the tile
      wave_lds_sync();
#pragma unroll
      for (int r = 0; r < 4; ++r) W.at(J, K, drow<double>(lk, r), li) = acc[r];
    }
    __syncthreads();
    if (J + 1 == T) break;
    // trailing update W_KK' -= R_JK^T R_JK', J < K <= K'.  Lookahead: wave 0
    // updates tile (J+1, J+1) first and factors it while the other waves
    // update the rest.
    const int rem = T - J - 1;
    const int pairs = rem * (rem + 1) / 2;
    if (wave == 0) {
      trail(J, J + 1, J + 1);
      // the tile just written is read back by other lanes of this wave
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      factor_diag(J + 1);
    } else {
      for (int pi = wave; pi < pairs; pi += nw - 1) {
        int a_ = 0, q = pi;
        while (q >= rem - a_) {
          q -= rem - a_;
          ++a_;
        }
        trail(J, J + 1 + a_, J + 1 + a_ + q);
      }
    }
    __syncthreads();
  }
  // R64 and Rc: upper tiles of W, zeros below the diagonal (same element
  // walk; reads of W unconditional, from the mirrored tile below the
  // diagonal, so a batch overlaps)
  {
    int ci = tid / lp, cj = tid - (tid / lp) * lp;
    while (ci < lp) {
      double v[kLoadU];
      int ii[kLoadU], jj[kLoadU];
#pragma unroll
      for (int u = 0; u < kLoadU; ++u) {
        const int i = ci < lp ? ci : lp - 1, j = cj;
        ii[u] = ci;
        jj[u] = cj;
        const int I = i >> 4, J = j >> 4;
        const bool up = I <= J;
        const double w = W.at(up ? I : J, up ? J : I, (up ? i : j) & 15, (up ? j : i) & 15);
        v[u] = w * ((I < J || (I == J && (i & 15) <= (j & 15))) ? 1.0 : 0.0);
        advance(ci, cj);
      }
#pragma unroll
      for (int u = 0; u < kLoadU; ++u) {
        if (ii[u] < lp) {
          const int64_t idx = static_cast<int64_t>(ii[u]) * lp + jj[u];
          if (kLds || ii[u] > jj[u]) R64[idx] = v[u];
          Rc[idx] = static_cast<C>(v[u]);
        }
      }
    }
  }
  if (tid == 0) {
    if (retry) {
      if (bad || tr_bad) flag[1] = 1;
      flag[2] += 1;
    } else {
      flag[0] = bad;
    }
  }
}

// ============================================================ tall triangular solve

// Each wave owns 16 rows of a 16*nwave-row block; column tile K of Q needs
// R[0..K][K] (a 16-column strip of R) and the inverse of R's diagonal tile K,
// staged once per block in LDS and shared by its waves.  Blocks stride over
// the row blocks.  With colpart, each block also writes the FP64 column sums
// of the Q rows it produced (values as stored) to colpart[blockIdx.x][:].
template <typename T, typename C>
__global__ void trsm_tall_kernel(int64_t rows, int l, T* Y, int64_t ld, const C* Rc, const C* Dc,
                                 double* colpart) {
  using V = typename Acc4<C>::type;
  extern __shared__ char tsm[];
  const int lp = pad16(l), TT = lp / 16, lq = lp + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  double* colacc = reinterpret_cast<double*>(tsm);         // lp column sums of this block
  double* red = colacc + lp;                               // 4 x 16 wave partial sums
  C* Rs = reinterpret_cast<C*>(red + 64);                  // lp x 16 strip of R
  C* Ds = Rs + static_cast<int64_t>(lp) * 16;              // 16 x 16 inverse tile
  C* Qs = Ds + 256 + static_cast<int64_t>(wave) * 16 * lq; // this wave's 16 rows of Q
  for (int c = threadIdx.x; c < lp; c += blockDim.x) colacc[c] = 0.0;
  const int64_t nblk = (rows + 16 * nwave - 1) / (16 * nwave);
  for (int64_t bt = blockIdx.x; bt < nblk; bt += gridDim.x) {
    const int64_t row0 = (bt * nwave + wave) * 16;
    for (int K = 0; K < TT; ++K) {
      const int col = K * 16 + li;
      V acc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + drow<C>(lk, r);
        acc[r] = (row < rows && col < l) ? ld_as<C>(Y + row * ld + col) : C(0);
      }
      __syncthreads();  // previous strip no longer in use
      for (int f = threadIdx.x; f < (K + 1) * 256; f += blockDim.x) {
        const int r = f >> 4, c = f & 15;
        Rs[f] = Rc[static_cast<int64_t>(r) * lp + K * 16 + c];
      }
      for (int f = threadIdx.x; f < 256; f += blockDim.x) Ds[f] = Dc[K * 256 + f];
      __syncthreads();
      for (int J = 0; J < K; ++J) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const C a = Qs[li * lq + J * 16 + kk * 4 + lk];
          const C b = Rs[(J * 16 + kk * 4 + lk) * 16 + li];
          acc = mfma4(-a, b, acc);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) Qs[drow<C>(lk, r) * lq + K * 16 + li] = acc[r];
      wave_lds_sync();
      V q = V{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) q = mfma4(Qs[li * lq + K * 16 + kk * 4 + lk], Ds[(kk * 4 + lk) * 16 + li], q);
      wave_lds_sync();
      double cs = 0.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Qs[drow<C>(lk, r) * lq + K * 16 + li] = q[r];
        const int64_t row = row0 + drow<C>(lk, r);
        if (row < rows && col < l) {
          T* dst = Y + row * ld + col;
          Elem<T>::store(dst, q[r]);
          if (colpart) cs += static_cast<double>(Elem<T>::load(dst));
        }
      }
      wave_lds_sync();
      if (colpart) {
        cs += __shfl_xor(cs, 16, 64);
        cs += __shfl_xor(cs, 32, 64);
        if (lk == 0) red[wave * 16 + li] = cs;
        __syncthreads();
        if (threadIdx.x < 16) {
          double t = 0.0;
          for (int w = 0; w < nwave; ++w) t += red[w * 16 + threadIdx.x];
          colacc[K * 16 + threadIdx.x] += t;
        }
      }
    }
  }
  if (colpart) {
    __syncthreads();
    for (int c = threadIdx.x; c < l; c += blockDim.x) colpart[static_cast<int64_t>(blockIdx.x) * l + c] = colacc[c];
  }
}

__global__ void upper_mult_kernel(int lp, const double* A, const double* B, double* Cm, int64_t ld) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(lp) * lp) return;
  const int i = static_cast<int>(idx / lp), j = static_cast<int>(idx % lp);
  double s = 0.0;
  for (int k = i; k <= j; ++k) s += A[static_cast<int64_t>(i) * ld + k] * B[static_cast<int64_t>(k) * ld + j];
  Cm[static_cast<int64_t>(i) * ld + j] = (i <= j) ? s : 0.0;
}

// ============================================================ tall Y <- Y R^-1, rows in registers

// Transposed form: the column tiles of Q = Y R^-1 satisfy
//   Q_K^T = D_K^T (Y_K^T - sum_{J<K} R_JK^T Q_J^T),   D_K = (R_KK)^-1,
// an MFMA problem in which every Q_J^T is a B operand.  The MFMA accumulator
// layout (lane (li, lk), value r holds row drow(lk, r), column li) is the B
// operand layout for k-step kk = r under the k-index order k = drow(lk, kk),
// so each output tile serves as an operand of the later tiles straight from
// registers, and lane (li, lk) reads and writes elements drow(lk, 0..3) of
// row li of its 16-row tile (four consecutive FP32 values).
//
// The A operands -R_JK^T and D_K^T are packed once per factor: tiles (J, K),
// J <= K, column tile by column tile (tile index K (K + 1) / 2 + J), 256
// entries each, entry (16 lk + li) 4 + kk holding -R[16 J + drow(lk, kk)][16 K + li]
// (J < K, negated so that the MFMAs subtract with no extra instruction) or
// D_K[drow(lk, kk)][li] (J = K): one 16-byte read per lane gives the four
// k-steps.
template <typename C>
__global__ void rfrag_pack_kernel(int lp, const double* R, const double* Dinv, C* Rf) {
  const int TT = lp / 16;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(TT) * (TT + 1) / 2 * 256) return;
  const int t = static_cast<int>(idx >> 8), e = static_cast<int>(idx & 255);
  int K = 0;
  while ((K + 1) * (K + 2) / 2 <= t) ++K;
  const int J = t - K * (K + 1) / 2;
  const int kk = e & 3, li = (e >> 2) & 15, lk = e >> 6;
  const int a = drow<C>(lk, kk);
  const double v = (J < K) ? -R[static_cast<int64_t>(16 * J + a) * lp + 16 * K + li] : Dinv[K * 256 + a * 16 + li];
  Rf[idx] = static_cast<C>(v);
}

// The value an element takes once stored in T.
template <typename T, typename C> __device__ inline C stored_as(C v) { return v; }
template <> __device__ inline float stored_as<bf16, float>(float v) { return bf16_to_float(float_to_bf16(v)); }

// Elements drow(lk, 0..3) of tile K of one row (zeros past `cols` or when !ok),
// as loaded: for BF16 storage v[0], v[1] hold the two 32-bit words of the four
// elements (packed in order) and widen_tile_row turns them into FP32 when the
// tile is used, so a look-ahead load does not wait at the point it is issued.
template <typename T, typename C>
__device__ inline void load_tile_row(const T* rowp, int K, int lk, int cols, bool ok, bool vec, C (&v)[4]) {
  if constexpr (std::is_same<T, bf16>::value) {
    const int c0 = 16 * K + 4 * lk;   // drow<float>(lk, r) = 4 lk + r
    if (ok && vec && c0 + 3 < cols) {
      const uint2 q = *reinterpret_cast<const uint2*>(rowp + c0);
      v[0] = __uint_as_float(q.x);
      v[1] = __uint_as_float(q.y);
    } else {
      uint32_t e[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) e[r] = (ok && c0 + r < cols) ? rowp[c0 + r].bits : 0u;
      v[0] = __uint_as_float(e[0] | (e[1] << 16));
      v[1] = __uint_as_float(e[2] | (e[3] << 16));
    }
    v[2] = v[3] = C(0);
    return;
  }
  if constexpr (!std::is_same<C, double>::value) {
    const int c0 = 16 * K + 4 * lk;
    if (ok && vec && c0 + 3 < cols) {
      const float4 q = *reinterpret_cast<const float4*>(rowp + c0);
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
      return;
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int c = 16 * K + drow<C>(lk, r);
    v[r] = (ok && c < cols) ? ld_as<C>(rowp + c) : C(0);
  }
}

// The values of a tile row left by load_tile_row (identity except for BF16).
template <typename T, typename C>
__device__ inline void widen_tile_row(C (&v)[4]) {
  if constexpr (std::is_same<T, bf16>::value) {
    const uint32_t w0 = __float_as_uint(v[0]), w1 = __float_as_uint(v[1]);
    v[0] = __uint_as_float(w0 << 16);
    v[1] = __uint_as_float(w0 & 0xffff0000u);
    v[2] = __uint_as_float(w1 << 16);
    v[3] = __uint_as_float(w1 & 0xffff0000u);
  }
}

// Four FP32 values rounded to BF16 (to nearest, ties to even), as two words
// of two elements each (element 0 in the low half of a).
__device__ inline void bf16_pack4(const float (&v)[4], uint32_t& a, uint32_t& b) {
  a = float2_to_bf16x2(v[0], v[1]);
  b = float2_to_bf16x2(v[2], v[3]);
}

template <typename T, typename C>
__device__ inline void store_tile_row(T* rowp, int K, int lk, int cols, bool ok, bool vec, const C (&v)[4]) {
  if (!ok) return;
  if constexpr (!std::is_same<C, double>::value) {
    const int c0 = 16 * K + 4 * lk;
    if (vec && c0 + 3 < cols) {
      if constexpr (std::is_same<T, float>::value) {
        *reinterpret_cast<float4*>(rowp + c0) = make_float4(v[0], v[1], v[2], v[3]);
      } else {
        uint32_t a, b;
        bf16_pack4(v, a, b);
        *reinterpret_cast<uint2*>(rowp + c0) = make_uint2(a, b);
      }
      return;
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int c = 16 * K + drow<C>(lk, r);
    if (c < cols) Elem<T>::store(rowp + c, v[r]);
  }
}

template <typename C>
__device__ inline void load_frag4(const C* p, C (&b)[4]) {
  if constexpr (std::is_same<C, float>::value) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    b[0] = q.x; b[1] = q.y; b[2] = q.z; b[3] = q.w;
  } else {
    const double2 q0 = *reinterpret_cast<const double2*>(p);
    const double2 q1 = *reinterpret_cast<const double2*>(p + 2);
    b[0] = q0.x; b[1] = q0.y; b[2] = q1.x; b[3] = q1.y;
  }
}

constexpr int kRowsTrsmParts = 1024;

// Each wave owns 16 rows at a time and walks the column tiles K in order; the
// finished tiles Q_J^T stay in its registers as B operands.  The sum over J is
// split over four accumulators (independent MFMA chains).  Tile K of Y is read
// just before it is overwritten by Q_K.  With colpart, each block writes the
// FP64 column sums of the values it stored (per wave in LDS, then in a fixed
// order over the waves).
template <typename T, typename C, int MT, bool STAGED>
__global__ __launch_bounds__(256) void trsm_rows_kernel(int64_t rows, int l, T* Y, int64_t ld, int vec,
                                                        const C* Rf_global, double* colpart) {
  using V = typename Acc4<C>::type;
  // FP32 blocks of at most 192 columns keep per-lane column sums of their rows
  // in registers and reduce them once; otherwise each tile is reduced at once
  constexpr bool REGSUM = std::is_same<C, float>::value && MT <= 12;
  C csl[REGSUM ? MT : 1][4];
#pragma unroll
  for (int J = 0; J < (REGSUM ? MT : 1); ++J)
#pragma unroll
    for (int r = 0; r < 4; ++r) csl[J][r] = C(0);
  __shared__ double csw[4][16 * MT];
  extern __shared__ __align__(16) unsigned char trsm_smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int TT = (l + 15) / 16;
  if (colpart) {
    for (int c = lane; c < 16 * MT; c += 64) csw[wave][c] = 0.0;
  }
  // STAGED: the packed factor (all TT (TT + 1) / 2 tiles) is copied to LDS once
  // per workgroup, so each column tile's operands come at LDS latency
  const C* Rf = Rf_global;
  if constexpr (STAGED) {
    C* lds = reinterpret_cast<C*>(trsm_smem);
    const int n4 = TT * (TT + 1) / 2 * 256 / 4;
    for (int f = threadIdx.x; f < n4; f += blockDim.x) {
      if constexpr (std::is_same<C, float>::value)
        reinterpret_cast<float4*>(lds)[f] = reinterpret_cast<const float4*>(Rf_global)[f];
      else {
        reinterpret_cast<double2*>(lds)[2 * f] = reinterpret_cast<const double2*>(Rf_global)[2 * f];
        reinterpret_cast<double2*>(lds)[2 * f + 1] = reinterpret_cast<const double2*>(Rf_global)[2 * f + 1];
      }
    }
    __syncthreads();
    Rf = lds;
  }
  if constexpr (MT <= 12) {
    const int64_t ntiles = (rows + 15) / 16;
    const int64_t tstride = static_cast<int64_t>(gridDim.x) * 4;
    // yb[K]: tile K of the current row tile of Y.  Once consumed it is refilled
    // with tile K of the wave's next row tile, so a whole row tile of loads is
    // in flight while the current one is solved.  Prefetch rows are clamped to
    // the last row (always valid addresses); stores stay masked.
    C yb[MT][4];
    int64_t rt = static_cast<int64_t>(blockIdx.x) * 4 + wave;
    {
      const int64_t r = (rt < ntiles ? rt : 0) * 16 + li;
      const T* rowp = Y + (r < rows ? r : rows - 1) * ld;
  #pragma unroll
      for (int K = 0; K < MT; ++K)
        if (K < TT && rows > 0) load_tile_row<T, C>(rowp, K, lk, l, true, vec != 0, yb[K]);
    }
    for (; rt < ntiles; rt += tstride) {
      const int64_t row0 = rt * 16;
      const bool rok = row0 + li < rows;
      T* rowp = Y + (row0 + li) * ld;
      const int64_t nr = (rt + tstride < ntiles ? rt + tstride : rt) * 16 + li;
      const T* nrowp = Y + (nr < rows ? nr : rows - 1) * ld;
      C q[MT][4];
  #pragma unroll
      for (int K = 0; K < MT; ++K) {
        if (K >= TT) continue;
        C y[4] = {yb[K][0], yb[K][1], yb[K][2], yb[K][3]};
        widen_tile_row<T, C>(y);
        load_tile_row<T, C>(nrowp, K, lk, l, true, vec != 0, yb[K]);
        V acc[4];
        acc[0] = V{y[0], y[1], y[2], y[3]};
        acc[1] = acc[2] = acc[3] = V{0, 0, 0, 0};
        const C* rk = Rf + static_cast<int64_t>(K * (K + 1) / 2) * 256 + 4 * lane;
  #pragma unroll
        for (int J = 0; J < K; ++J) {
          C a[4];
          load_frag4<C>(rk + 256 * J, a);
  #pragma unroll
          for (int kk = 0; kk < 4; ++kk) acc[J & 3] = mfma4(a[kk], q[J][kk], acc[J & 3]);
        }
        const V sacc = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        C d[4];
        load_frag4<C>(rk + 256 * K, d);
        V out = V{0, 0, 0, 0};
  #pragma unroll
        for (int kk = 0; kk < 4; ++kk) out = mfma4(d[kk], sacc[kk], out);
  #pragma unroll
        for (int r = 0; r < 4; ++r) q[K][r] = out[r];
        store_tile_row<T, C>(rowp, K, lk, l, rok, vec != 0, q[K]);
        if constexpr (REGSUM) {
          if (colpart) {
  #pragma unroll
            for (int r = 0; r < 4; ++r)
              if (rok && 16 * K + drow<C>(lk, r) < l) csl[K][r] += stored_as<T, C>(q[K][r]);
          }
        } else if (colpart) {
          double cs[4];
  #pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int c = 16 * K + drow<C>(lk, r);
            cs[r] = (rok && c < l) ? static_cast<double>(stored_as<T, C>(q[K][r])) : 0.0;
            cs[r] = row16_sum(cs[r]);   // DPP: no LDS traffic
          }
          if (li == 0) {
  #pragma unroll
            for (int r = 0; r < 4; ++r) csw[wave][16 * K + drow<C>(lk, r)] += cs[r];
          }
        }
      }
    }
  } else {
    // wider blocks (the register budget allows no more): one tile of
    // look-ahead for Y, carried across row tiles; the factor fragments of a
    // column tile are read kGroup at a time (clamped to valid tiles, so a
    // group's loads are in flight together)
    constexpr int kGroup = 4;
    const int64_t ntiles = (rows + 15) / 16;
    const int64_t tstride = static_cast<int64_t>(gridDim.x) * 4;
    int64_t rt = static_cast<int64_t>(blockIdx.x) * 4 + wave;
    C ynext[4] = {C(0), C(0), C(0), C(0)};
    if (rows > 0) {
      const int64_t r = (rt < ntiles ? rt : 0) * 16 + li;
      load_tile_row<T, C>(Y + (r < rows ? r : rows - 1) * ld, 0, lk, l, true, vec != 0, ynext);
    }
    for (; rt < ntiles; rt += tstride) {
      const int64_t row0 = rt * 16;
      const bool rok = row0 + li < rows;
      T* rowp = Y + (row0 + li) * ld;
      const T* crowp = Y + (rok ? row0 + li : rows - 1) * ld;
      const int64_t nr = (rt + tstride < ntiles ? rt + tstride : rt) * 16 + li;
      const T* nrowp = Y + (nr < rows ? nr : rows - 1) * ld;
      C q[MT][4];
#pragma unroll 1
      for (int K = 0; K < TT; ++K) {
        C y[4] = {ynext[0], ynext[1], ynext[2], ynext[3]};
        widen_tile_row<T, C>(y);
        if (K + 1 < TT) load_tile_row<T, C>(crowp, K + 1, lk, l, true, vec != 0, ynext);
        else load_tile_row<T, C>(nrowp, 0, lk, l, true, vec != 0, ynext);
        V acc[4];
        acc[0] = V{y[0], y[1], y[2], y[3]};
        acc[1] = acc[2] = acc[3] = V{0, 0, 0, 0};
        const C* rk = Rf + static_cast<int64_t>(K * (K + 1) / 2) * 256 + 4 * lane;
#pragma unroll
        for (int J0 = 0; J0 < MT; J0 += kGroup) {
          if (J0 >= K) continue;
          C a[kGroup][4];
#pragma unroll
          for (int g = 0; g < kGroup; ++g) load_frag4<C>(rk + 256 * (J0 + g < K ? J0 + g : J0), a[g]);
#pragma unroll
          for (int g = 0; g < kGroup; ++g) {
            if (J0 + g >= MT || J0 + g >= K) continue;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) acc[g & 3] = mfma4(a[g][kk], q[J0 + g][kk], acc[g & 3]);
          }
        }
        const V sacc = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        C d[4];
        load_frag4<C>(rk + 256 * K, d);
        V out = V{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) out = mfma4(d[kk], sacc[kk], out);
        C o[4] = {out[0], out[1], out[2], out[3]};
#pragma unroll
        for (int J = 0; J < MT; ++J)
          if (J == K) {
#pragma unroll
            for (int r = 0; r < 4; ++r) q[J][r] = o[r];
          }
        store_tile_row<T, C>(rowp, K, lk, l, rok, vec != 0, o);
        if constexpr (REGSUM) {
          if (colpart) {
#pragma unroll
            for (int J = 0; J < MT; ++J)
              if (J == K) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                  if (rok && 16 * K + drow<C>(lk, r) < l) csl[J][r] += stored_as<T, C>(o[r]);
              }
          }
        } else if (colpart) {
          double cs[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int c = 16 * K + drow<C>(lk, r);
            cs[r] = (rok && c < l) ? static_cast<double>(stored_as<T, C>(o[r])) : 0.0;
            cs[r] = row16_sum(cs[r]);   // DPP: no LDS traffic
          }
          if (li == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) csw[wave][16 * K + drow<C>(lk, r)] += cs[r];
          }
        }
      }
    }
  }
  if (colpart) {
    if constexpr (REGSUM) {
      // one reduction over the 16 rows of the lane groups, in FP64
#pragma unroll
      for (int J = 0; J < MT; ++J) {
        if (J < TT) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double v = static_cast<double>(csl[J][r]);
            v = row16_sum(v);
            if (li == 0) csw[wave][16 * J + drow<C>(lk, r)] = v;
          }
        }
      }
    }
    __syncthreads();
    for (int col = threadIdx.x; col < l; col += blockDim.x)
      colpart[static_cast<int64_t>(blockIdx.x) * l + col] = (csw[0][col] + csw[1][col]) + (csw[2][col] + csw[3][col]);
  }
}

// Wide FP32 solve for blocks of exactly 16 MT columns (MT = 16 or 18), rows
// 16-byte aligned: the off-diagonal tiles of the packed factor (MT (MT - 1) / 2
// KiB; 153 KiB at l = 288) are copied once into the LDS of a persistent
// workgroup of W waves, one workgroup per CU; the diagonal inverses come from
// global memory (L2), one tile ahead of use.  A wave walks 16-row tiles as
// trsm_rows_kernel does.  Y is read through a ring of MT / 2 tile slots:
// consuming tile K of the current row tile frees slot K mod MT / 2, which
// receives tile K + MT / 2 of the same row tile or, in the second half, tile
// K - MT / 2 of the wave's next row tile.  Every access is a whole 16-byte
// (FP32) or 8-byte (BF16) word; only stores of rows past the end are masked.
// Column sums: after each column tile the 16 rows' values are summed in FP64
// across the lanes of a column (shuffles) and lane li keeps the sums of the
// tiles K with K mod 16 == li.
template <typename T> __device__ inline void load_full_tile(const T* rowp, int K, int lk, float (&v)[4]);
template <> __device__ inline void load_full_tile<float>(const float* rowp, int K, int lk, float (&v)[4]) {
  const float4 q = *reinterpret_cast<const float4*>(rowp + 16 * K + 4 * lk);
  v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
}
template <> __device__ inline void load_full_tile<bf16>(const bf16* rowp, int K, int lk, float (&v)[4]) {
  const uint2 q = *reinterpret_cast<const uint2*>(rowp + 16 * K + 4 * lk);
  v[0] = __uint_as_float(q.x);   // two packed words, widened by widen_tile_row
  v[1] = __uint_as_float(q.y);
  v[2] = v[3] = 0.f;
}

template <typename T, int MT, int W>
__global__ __launch_bounds__(64 * W) void trsm_wide_kernel(int64_t rows, T* Y, int64_t ld, const float* Rf,
                                                           double* colpart) {
  using C = float;
  using V = v4f;
  constexpr int H = MT / 2;   // ring slots
  constexpr int L = 16 * MT;
  extern __shared__ __align__(16) unsigned char trsm_smem[];
  float* off = reinterpret_cast<float*>(trsm_smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  {
    // LDS tile K (K - 1) / 2 + J  <-  packed tile K (K + 1) / 2 + J, J < K
    constexpr int n16 = MT * (MT - 1) / 2 * 64;
    for (int f = threadIdx.x; f < n16; f += blockDim.x) {
      const int t = f >> 6, e = f & 63;
      int K = 1;
      while (K * (K + 1) / 2 <= t) ++K;
      const int J = t - K * (K - 1) / 2;
      reinterpret_cast<float4*>(off)[f] =
          reinterpret_cast<const float4*>(Rf + static_cast<int64_t>(K * (K + 1) / 2 + J) * 256)[e];
    }
    __syncthreads();
  }
  // column sums: lane li keeps column 4 lk + row16_sum4_index(li) of the tiles
  // K with K mod 4 = li / 4
  constexpr int NS4 = (MT + 3) / 4;
  double cacc[NS4];
#pragma unroll
  for (int s2 = 0; s2 < NS4; ++s2) cacc[s2] = 0.0;
  const int64_t ntiles = (rows + 15) / 16;
  const int64_t tstride = static_cast<int64_t>(gridDim.x) * W;
  int64_t rt = static_cast<int64_t>(blockIdx.x) * W + wave;
  auto clamp_row = [&](int64_t tile) {
    const int64_t r = tile * 16 + li;
    return Y + (r < rows ? r : rows - 1) * ld;
  };
  C yb[H][4];
  {
    const T* rowp = clamp_row(rt < ntiles ? rt : 0);
#pragma unroll
    for (int K = 0; K < H; ++K) load_full_tile<T>(rowp, K, lk, yb[K]);
  }
  for (; rt < ntiles; rt += tstride) {
    const int64_t row0 = rt * 16;
    const bool rok = row0 + li < rows;
    T* rowp = Y + (row0 + li) * ld;
    const T* crowp = clamp_row(rt);
    const T* nrowp = clamp_row(rt + tstride < ntiles ? rt + tstride : rt);
    C q[MT][4];
    C dn[4];
    load_frag4<C>(Rf + 4 * lane, dn);   // D_0 (packed tile 0)
#pragma unroll
    for (int K = 0; K < MT; ++K) {
      C d[4] = {dn[0], dn[1], dn[2], dn[3]};
      if (K + 1 < MT) load_frag4<C>(Rf + static_cast<int64_t>((K + 1) * (K + 4) / 2) * 256 + 4 * lane, dn);
      C y[4] = {yb[K % H][0], yb[K % H][1], yb[K % H][2], yb[K % H][3]};
      widen_tile_row<T, C>(y);
      if (K + H < MT) load_full_tile<T>(crowp, K + H, lk, yb[K % H]);
      else load_full_tile<T>(nrowp, K + H - MT, lk, yb[K % H]);
      V acc[4];
      acc[0] = V{y[0], y[1], y[2], y[3]};
      acc[1] = acc[2] = acc[3] = V{0, 0, 0, 0};
      const float* rk = off + (K * (K - 1) / 2) * 256 + 4 * lane;
      // tiles J of a group of four feed the four accumulators in turn, so
      // consecutive MFMAs never depend on each other; the next group's factor
      // fragments are read from LDS while the current group's MFMAs run (one
      // group ahead only: the scheduling barrier keeps the registers bounded)
      C a[4][4];
#pragma unroll
      for (int g = 0; g < 4; ++g)
        if (g < K) load_frag4<C>(rk + 256 * g, a[g]);
#pragma unroll
      for (int J0 = 0; J0 < K; J0 += 4) {
        C an[4][4];
#pragma unroll
        for (int g = 0; g < 4; ++g)
          if (J0 + 4 + g < K) load_frag4<C>(rk + 256 * (J0 + 4 + g), an[g]);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
          for (int g = 0; g < 4; ++g)
            if (J0 + g < K) acc[g] = mfma4(a[g][kk], q[J0 + g][kk], acc[g]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) a[g][kk] = an[g][kk];
      }
      const V sacc = (acc[0] + acc[1]) + (acc[2] + acc[3]);
      // D_K^T applied with two accumulators (k-steps 0, 1 and 2, 3)
      V out = V{0, 0, 0, 0}, out2 = V{0, 0, 0, 0};
      out = mfma4(d[0], sacc[0], out);
      out2 = mfma4(d[2], sacc[2], out2);
      out = mfma4(d[1], sacc[1], out);
      out2 = mfma4(d[3], sacc[3], out2);
      out += out2;
#pragma unroll
      for (int r = 0; r < 4; ++r) q[K][r] = out[r];
      // the stored values (BF16: rounded once, for the store and the sums)
      double cs[4];
      if constexpr (std::is_same<T, bf16>::value) {
        uint32_t wa, wb;
        bf16_pack4(q[K], wa, wb);
        if (rok) *reinterpret_cast<uint2*>(rowp + 16 * K + 4 * lk) = make_uint2(wa, wb);
        cs[0] = __uint_as_float(wa << 16);
        cs[1] = __uint_as_float(wa & 0xffff0000u);
        cs[2] = __uint_as_float(wb << 16);
        cs[3] = __uint_as_float(wb & 0xffff0000u);
      } else {
        store_tile_row<T, C>(rowp, K, lk, L, rok, true, q[K]);
#pragma unroll
        for (int r = 0; r < 4; ++r) cs[r] = q[K][r];
      }
      if (colpart) {
#pragma unroll
        for (int r = 0; r < 4; ++r) cs[r] = rok ? cs[r] : 0.0;
        const double s = row16_sum4(cs, li);   // DPP: no LDS traffic
        if ((li >> 2) == (K & 3)) cacc[K >> 2] += s;
      }
    }
  }
  if (colpart) {
    __syncthreads();   // every wave is done with the factor: its LDS takes the sums
    double* csw = reinterpret_cast<double*>(trsm_smem);
#pragma unroll
    for (int s2 = 0; s2 < NS4; ++s2) {
      const int K = 4 * s2 + (li >> 2);
      if (K < MT) csw[wave * L + 16 * K + drow<C>(lk, row16_sum4_index(li))] = cacc[s2];
    }
    __syncthreads();
    for (int col = threadIdx.x; col < L; col += blockDim.x) {
      double v = 0.0;
      for (int w = 0; w < W; ++w) v += csw[w * L + col];
      colpart[static_cast<int64_t>(blockIdx.x) * L + col] = v;
    }
  }
}

__global__ void zero_doubles_kernel(int64_t n, double* x) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx < n) x[idx] = 0.0;
}

// ============================================================ one-sided Jacobi SVD

constexpr int kJacobiMaxN = 1024;
constexpr int kJacobiPerLane = 22;   // column elements per lane of a pair group

// One-sided (Hestenes) Jacobi on the columns of A, round-robin ("circle")
// pair ordering: in each of the np-1 rounds every column is in exactly one
// pair, pairs are independent.  A group of G lanes owns one pair: both
// columns sit in its registers (kJacobiPerLane elements per lane), so a round
// costs one round trip to memory; the rotation accumulator rows are touched
// only when the pair is rotated.
template <int G>
__global__ __launch_bounds__(1024) void jacobi_kernel(int n, const double* A, int64_t lda, double* Uo,
                                                      double* s, double* Vo, double* work, int* sweeps_out) {
  const int np = n + (n & 1);
  double* Wt = work;                                   // np x n : column p of A as row p
  double* Jt = work + static_cast<int64_t>(np) * n;    // np x n : accumulated rotations
  double* sig = Jt + static_cast<int64_t>(np) * n;     // np
  int* rank = reinterpret_cast<int*>(sig + np);        // np
  const int tid = threadIdx.x;
  const int grp = tid / G, gl = tid % G, ngrp = blockDim.x / G;
  __shared__ int rotated;
  for (int64_t idx = tid; idx < static_cast<int64_t>(np) * n; idx += blockDim.x) {
    const int p = static_cast<int>(idx / n), i = static_cast<int>(idx % n);
    Wt[idx] = p < n ? A[static_cast<int64_t>(i) * lda + p] : 0.0;
    Jt[idx] = (p == i) ? 1.0 : 0.0;
  }
  __syncthreads();
  // rotate while |cos| of the column pair exceeds n eps (below that the pair
  // is orthogonal to working accuracy)
  const double tol = static_cast<double>(n) * 2.220446049250313e-16;
  int sweep = 0;
  for (; sweep < 60; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < np - 1; ++r) {
      for (int k = grp; k < np / 2; k += ngrp) {
        const int a = (k == 0) ? 0 : ((k - 1 + r) % (np - 1)) + 1;
        const int b = ((np - 2 - k + r) % (np - 1)) + 1;
        double* wa = Wt + static_cast<int64_t>(a) * n;
        double* wb = Wt + static_cast<int64_t>(b) * n;
        double x[kJacobiPerLane], y[kJacobiPerLane];
#pragma unroll
        for (int e = 0; e < kJacobiPerLane; ++e) {
          const int i = gl + G * e;
          x[e] = i < n ? wa[i] : 0.0;
          y[e] = i < n ? wb[i] : 0.0;
        }
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int e = 0; e < kJacobiPerLane; ++e) {
          al += x[e] * x[e];
          be += y[e] * y[e];
          ga += x[e] * y[e];
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
          al += __shfl_xor(al, off, G);
          be += __shfl_xor(be, off, G);
          ga += __shfl_xor(ga, off, G);
        }
        if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          const double sn = c * t;
          double* ja = Jt + static_cast<int64_t>(a) * n;
          double* jb = Jt + static_cast<int64_t>(b) * n;
#pragma unroll
          for (int e = 0; e < kJacobiPerLane; ++e) {
            const int i = gl + G * e;
            if (i < n) {
              wa[i] = c * x[e] - sn * y[e];
              wb[i] = sn * x[e] + c * y[e];
            }
          }
          // accumulator rows in chunks of 8 elements per lane (register budget)
#pragma unroll
          for (int e0 = 0; e0 < kJacobiPerLane; e0 += 8) {
            double u[8], v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int i = gl + G * (e0 + e);
              u[e] = (e0 + e < kJacobiPerLane && i < n) ? ja[i] : 0.0;
              v[e] = (e0 + e < kJacobiPerLane && i < n) ? jb[i] : 0.0;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int i = gl + G * (e0 + e);
              if (e0 + e < kJacobiPerLane && i < n) {
                ja[i] = c * u[e] - sn * v[e];
                jb[i] = sn * u[e] + c * v[e];
              }
            }
          }
          if (gl == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  for (int p = grp; p < np; p += ngrp) {
    const double* wp = Wt + static_cast<int64_t>(p) * n;
    double acc = 0.0;
    for (int i = gl; i < n; i += G) acc += wp[i] * wp[i];
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
    if (gl == 0) sig[p] = sqrt(acc);
  }
  __syncthreads();
  for (int p = tid; p < n; p += blockDim.x) {
    const double sp = sig[p];
    int rk = 0;
    for (int q = 0; q < n; ++q) {
      const double sq = sig[q];
      rk += (sq > sp || (sq == sp && q < p)) ? 1 : 0;
    }
    rank[p] = rk;
    s[rk] = sp;
  }
  __syncthreads();
  for (int64_t idx = tid; idx < static_cast<int64_t>(n) * n; idx += blockDim.x) {
    const int p = static_cast<int>(idx / n), i = static_cast<int>(idx % n);
    const int rk = rank[p];
    const double sp = sig[p];
    Uo[static_cast<int64_t>(i) * n + rk] = sp > 0.0 ? Wt[idx] / sp : 0.0;
    Vo[static_cast<int64_t>(i) * n + rk] = Jt[idx];
  }
  if (tid == 0 && sweeps_out) *sweeps_out = sweep;
}

// ---------------------------------------------------------------- block Jacobi
//
// Columns are grouped in blocks of B; each launch is one round of the
// round-robin over blocks, one workgroup per block pair.  A workgroup loads
// its 2B columns of W (and the matching rows of the rotation accumulator J)
// into LDS and runs one full one-sided Jacobi sweep among them (2B-1 inner
// rounds of B independent pairs).  A pair is owned by one row of 16 lanes:
// each lane holds PER >= ceil(n/16) elements of both columns in registers
// for the inner round and the three 16-lane sums go through DPP, so an inner
// round costs one LDS round trip and one barrier.  Columns sit in LDS with
// stride 16 PER, zero beyond n, so every access is unconditional (rotating
// zeros keeps them zero).  flags[0] = converged (every
// later launch returns at once), flags[1 + s] = rotated in sweep s.

template <int B, int PER>
__global__ __launch_bounds__(16 * B) void bjacobi_round_kernel(int n, int nb, int round, int sweep, double* Wt,
                                                               double* Jt, int* flags, double rel_tol) {
  if (flags[0]) return;
  extern __shared__ double bjs[];
  constexpr int NS = 16 * PER;    // LDS column stride
  double* Ws = bjs;               // 2B columns
  double* Js = bjs + 2 * B * NS;  // 2B columns
  __shared__ int any_rot;
  const int w = blockIdx.x;
  const int pa = (w == 0) ? 0 : ((w - 1 + round) % (nb - 1)) + 1;
  const int pb = ((nb - 2 - w + round) % (nb - 1)) + 1;
  // 2 PER elements of W and of J per thread, all loads in flight together
  constexpr int kCopy = 2 * PER;
  auto copy_index = [&](int j, int& f, int64_t& gidx, bool& in) {
    f = threadIdx.x + j * 16 * B;
    const int lc = f / NS, i = f - lc * NS;
    gidx = (static_cast<int64_t>(lc < B ? pa : pb) * B + (lc & (B - 1))) * n + i;
    in = i < n;
  };
  {
    double wv[kCopy], jv[kCopy];
#pragma unroll
    for (int j = 0; j < kCopy; ++j) {
      int f;
      int64_t gi;
      bool in;
      copy_index(j, f, gi, in);
      wv[j] = in ? Wt[gi] : 0.0;
      jv[j] = in ? Jt[gi] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kCopy; ++j) {
      const int f = threadIdx.x + j * 16 * B;
      Ws[f] = wv[j];
      Js[f] = jv[j];
    }
  }
  if (threadIdx.x == 0) any_rot = 0;
  __syncthreads();
  // rotate while |cos| of the column pair exceeds rel_tol (default n eps)
  const double tol = rel_tol > 0.0 ? rel_tol : static_cast<double>(n) * 2.220446049250313e-16;
  constexpr int P = 2 * B;      // local players
  constexpr bool kPreJ = PER <= 20;  // J rows loaded with W's (register budget)
  const int k = threadIdx.x >> 4, g = threadIdx.x & 15;
  int rot = 0;
  for (int r = 0; r < P - 1; ++r) {
    const int a = (k == 0) ? 0 : ((k - 1 + r) % (P - 1)) + 1;
    const int b = ((P - 2 - k + r) % (P - 1)) + 1;
    double* wa = Ws + a * NS + g;
    double* wb = Ws + b * NS + g;
    double* ja = Js + a * NS + g;
    double* jb = Js + b * NS + g;
    double x[PER], y[PER], u[PER], v[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      x[e] = wa[16 * e];
      y[e] = wb[16 * e];
      if (kPreJ) {
        u[e] = ja[16 * e];
        v[e] = jb[16 * e];
      }
    }
    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      al += x[e] * x[e];
      be += y[e] * y[e];
      ga += x[e] * y[e];
    }
    al = row16_sum(al);
    be = row16_sum(be);
    ga = row16_sum(ga);
    if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
      const double zeta = (be - al) / (2.0 * ga);
      const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
      const double c = 1.0 / sqrt(1.0 + t * t);
      const double sn = c * t;
      if (!kPreJ) {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
          u[e] = ja[16 * e];
          v[e] = jb[16 * e];
        }
      }
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        wa[16 * e] = c * x[e] - sn * y[e];
        wb[16 * e] = sn * x[e] + c * y[e];
        ja[16 * e] = c * u[e] - sn * v[e];
        jb[16 * e] = sn * u[e] + c * v[e];
      }
      rot = 1;
    }
    __syncthreads();
  }
  if (rot) any_rot = 1;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kCopy; ++j) {
    int f;
    int64_t gi;
    bool in;
    copy_index(j, f, gi, in);
    if (in) {
      Wt[gi] = Ws[f];
      Jt[gi] = Js[f];
    }
  }
  if (threadIdx.x == 0 && any_rot) flags[1 + sweep] = 1;
}

// Row p of Wt = column p of A V0, row p of Jt = column p of V0 (V0 = I when
// absent): the sweeps then rotate A V0, and the accumulated rotation starts at
// V0, so a V0 close to A's right singular vectors saves sweeps and any
// orthogonal V0 gives the same decomposition.
__global__ void bjacobi_init_kernel(int n, int np, const double* A, int64_t lda, const double* V0, double* Wt,
                                    double* Jt, int* flags, int nflags) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx < nflags) flags[idx] = 0;
  if (idx >= static_cast<int64_t>(np) * n) return;
  const int p = static_cast<int>(idx / n), i = static_cast<int>(idx % n);
  if (V0 == nullptr) {
    Wt[idx] = p < n ? A[static_cast<int64_t>(i) * lda + p] : 0.0;
    Jt[idx] = (p == i) ? 1.0 : 0.0;
  } else if (p < n) {
    double w = 0.0;
    for (int q = 0; q < n; ++q) w += A[static_cast<int64_t>(i) * lda + q] * V0[static_cast<int64_t>(q) * n + p];
    Wt[idx] = w;
    Jt[idx] = V0[static_cast<int64_t>(i) * n + p];
  } else {
    Wt[idx] = 0.0;
    Jt[idx] = 0.0;
  }
}

__global__ void bjacobi_check_kernel(int sweep, int* flags) {
  if (threadIdx.x == 0 && !flags[0] && !flags[1 + sweep]) {
    flags[0] = 1;
    flags[1 + 64] = sweep;  // sweeps taken (the last one rotated nothing)
  }
}

// Singular values (column norms), descending order, U = W / s, V = J.
__global__ __launch_bounds__(1024) void bjacobi_finish_kernel(int n, const double* Wt, const double* Jt, double* Uo,
                                                             double* s, double* Vo, double* sig, int* rank,
                                                             const int* flags, int* sweeps_out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int p = wave; p < n; p += nw) {
    double acc = 0.0;
    for (int i = lane; i < n; i += 64) {
      const double x = Wt[static_cast<int64_t>(p) * n + i];
      acc += x * x;
    }
    acc = wave_sum(acc);
    if (lane == 0) sig[p] = sqrt(acc);
  }
  __syncthreads();
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    const double sp = sig[p];
    int rk = 0;
    for (int q = 0; q < n; ++q) {
      const double sq = sig[q];
      rk += (sq > sp || (sq == sp && q < p)) ? 1 : 0;
    }
    rank[p] = rk;
    s[rk] = sp;
  }
  __syncthreads();
  for (int64_t idx = threadIdx.x; idx < static_cast<int64_t>(n) * n; idx += blockDim.x) {
    const int p = static_cast<int>(idx / n), i = static_cast<int>(idx % n);
    const int rk = rank[p];
    const double sp = sig[p];
    Uo[static_cast<int64_t>(i) * n + rk] = sp > 0.0 ? Wt[idx] / sp : 0.0;
    Vo[static_cast<int64_t>(i) * n + rk] = Jt[idx];
  }
  if (threadIdx.x == 0 && sweeps_out) *sweeps_out = flags[0] ? flags[1 + 64] + 1 : -1;
}

// ============================================================ Philox Gaussian

__device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = static_cast<uint64_t>(M0) * c[0];
    const uint64_t p1 = static_cast<uint64_t>(M1) * c[2];
    const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
    const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

template <typename T>
__global__ void gaussian_kernel(int64_t rows, int64_t cols, uint64_t seed, T* out, int64_t ld) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t total = rows * cols;
  if (2 * g >= total) return;
  uint32_t c[4] = {static_cast<uint32_t>(g), static_cast<uint32_t>(static_cast<uint64_t>(g) >> 32), 0u, 0u};
  philox10(c, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  const double two26 = 67108864.0, inv53 = 1.0 / 9007199254740992.0;
  const double u1 = ((c[0] >> 5) * two26 + (c[1] >> 6) + 0.5) * inv53;
  const double u2 = ((c[2] >> 5) * two26 + (c[3] >> 6) + 0.5) * inv53;
  const double rad = sqrt(-2.0 * log(u1));
  const double th = 6.283185307179586476925286766559 * u2;
  const double z[2] = {rad * cos(th), rad * sin(th)};
  for (int h = 0; h < 2; ++h) {
    const int64_t e = 2 * g + h;
    if (e >= total) break;
    const int64_t r = e / cols, cc = e % cols;
    Elem<T>::store(out + r * ld + cc, static_cast<typename ComputeOf<T>::type>(z[h]));
  }
}

template <typename D, typename S>
__global__ void convert_kernel(int64_t rows, int64_t cols, const S* src, int64_t lds, D* dst, int64_t ldd) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t r = idx / cols, c = idx % cols;
  using CD = typename ComputeOf<D>::type;
  Elem<D>::store(dst + r * ldd + c, static_cast<CD>(Elem<S>::load(src + r * lds + c)));
}

template <typename C>
__global__ void pack_residual_rhs_kernel(int l, int k, const double* UR, const double* ZR, const double* s,
                                         int64_t ld, C* B) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * l * k) return;
  const int r = idx / k, c = idx % k;
  const double v = r < l ? UR[static_cast<int64_t>(r) * ld + c] : -ZR[static_cast<int64_t>(r - l) * ld + c] * s[c];
  B[idx] = static_cast<C>(v);
}

__global__ void small_residual_kernel(int l, int k, const double* Rc, int64_t ldr, const double* ZR,
                                      const double* UR, int64_t ldu, const double* s, double* out) {
  const int i = blockIdx.x;
  if (i >= k) return;
  double acc = 0.0;
  for (int row = threadIdx.x; row < l; row += blockDim.x) {
    double v = 0.0;
    for (int c = row; c < l; ++c) v += Rc[static_cast<int64_t>(row) * ldr + c] * ZR[static_cast<int64_t>(c) * ldu + i];
    v -= s[i] * UR[static_cast<int64_t>(row) * ldu + i];
    acc += v * v;
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

}  // namespace

// ============================================================ host wrappers

size_t gram_workspace_doubles(int64_t rows, int m, int p) {
  const int64_t nparts = ceil_div(rows > 0 ? rows : 1, gram_rows_per_part(rows));
  return static_cast<size_t>(nparts) * pad16(m) * pad16(p);
}

template <typename T>
void launch_gram(int64_t rows, int m, int p, const T* A, int64_t lda, const T* B, int64_t ldb, bool same,
                 double* C, int64_t ldc, double* work, hipStream_t stream) {
  gram_impl<T, T>(rows, m, p, A, lda, B, ldb, same, C, ldc, work, stream);
}

int gram_max_parts_for(int m, int p, size_t work_doubles) {
  const size_t per_part = static_cast<size_t>(pad16(m)) * pad16(p);
  const size_t parts = per_part ? work_doubles / per_part : 0;
  return static_cast<int>(parts < static_cast<size_t>(kGramMaxParts) ? parts : kGramMaxParts);
}

template <typename T>
void launch_gram_bounded(int64_t rows, int m, int p, const T* A, int64_t lda, const T* B, int64_t ldb, bool same,
                         double* C, int64_t ldc, double* work, size_t work_doubles, hipStream_t stream) {
  const int parts = gram_max_parts_for(m, p, work_doubles);
  ISVD_CHECK(parts >= 1, ISVD_E_INVALID, "gram: the workspace cannot hold one row slice of the result");
  gram_impl<T, T>(rows, m, p, A, lda, B, ldb, same, C, ldc, work, stream, parts);
}
template void launch_gram_bounded<double>(int64_t, int, int, const double*, int64_t, const double*, int64_t, bool, double*, int64_t, double*, size_t, hipStream_t);
template void launch_gram_bounded<float>(int64_t, int, int, const float*, int64_t, const float*, int64_t, bool, double*, int64_t, double*, size_t, hipStream_t);
template void launch_gram_bounded<bf16>(int64_t, int, int, const bf16*, int64_t, const bf16*, int64_t, bool, double*, int64_t, double*, size_t, hipStream_t);
template <typename TA, typename TB>
void launch_gram2(int64_t rows, int m, int p, const TA* A, int64_t lda, const TB* B, int64_t ldb,
                  double* C, int64_t ldc, double* work, hipStream_t stream) {
  gram_impl<TA, TB>(rows, m, p, A, lda, B, ldb, false, C, ldc, work, stream);
}
template void launch_gram<double>(int64_t, int, int, const double*, int64_t, const double*, int64_t, bool, double*, int64_t, double*, hipStream_t);
template void launch_gram<float>(int64_t, int, int, const float*, int64_t, const float*, int64_t, bool, double*, int64_t, double*, hipStream_t);
template void launch_gram<bf16>(int64_t, int, int, const bf16*, int64_t, const bf16*, int64_t, bool, double*, int64_t, double*, hipStream_t);
template void launch_gram2<double, double>(int64_t, int, int, const double*, int64_t, const double*, int64_t, double*, int64_t, double*, hipStream_t);
template void launch_gram2<float, float>(int64_t, int, int, const float*, int64_t, const float*, int64_t, double*, int64_t, double*, hipStream_t);
template void launch_gram2<float, bf16>(int64_t, int, int, const float*, int64_t, const bf16*, int64_t, double*, int64_t, double*, hipStream_t);
template void launch_gram2<bf16, bf16>(int64_t, int, int, const bf16*, int64_t, const bf16*, int64_t, double*, int64_t, double*, hipStream_t);

size_t gemm_colnorm_workspace(int64_t M, int N) {
  (void)M;
  return static_cast<size_t>(kColnormParts) * N;
}

template <typename T>
void launch_gemm_tall(int64_t M, int N, int K1, const T* A1, int64_t lda1, int K2, const T* A2,
                      int64_t lda2, const typename ComputeOf<T>::type* B, int64_t ldb, T* Cm,
                      int64_t ldc, double alpha, double beta, GemmEpi epi, double* colnorm,
                      double* work, hipStream_t stream) {
  using C = typename ComputeOf<T>::type;
  if (M <= 0 || N <= 0) return;
  if constexpr (std::is_same<T, float>::value) {
    if (epi == GemmEpi::Store && K2 == 0 && beta == 0.0 &&
        gemm_rows_try(M, N, K1, A1, lda1, B, ldb, Cm, ldc, alpha, stream))
      return;
  }
  const int tiles = static_cast<int>(ceil_div(N, 16));
  const int ncb = static_cast<int>(ceil_div(tiles, 8));
  const int tn = static_cast<int>(ceil_div(tiles, ncb));
  switch (tn) {
#define ISVD_TN(X) \
  case X: return gemm_launch_tn<T, C, X>(M, N, K1, A1, lda1, K2, A2, lda2, B, ldb, Cm, ldc, alpha, beta, epi, colnorm, work, stream);
    ISVD_TN(1) ISVD_TN(2) ISVD_TN(3) ISVD_TN(4) ISVD_TN(5) ISVD_TN(6) ISVD_TN(7) ISVD_TN(8)
#undef ISVD_TN
    default: throw Error{ISVD_E_INVALID, "gemm: bad tile count"};
  }
}
template void launch_gemm_tall<double>(int64_t, int, int, const double*, int64_t, int, const double*, int64_t, const double*, int64_t, double*, int64_t, double, double, GemmEpi, double*, double*, hipStream_t);
template void launch_gemm_tall<float>(int64_t, int, int, const float*, int64_t, int, const float*, int64_t, const float*, int64_t, float*, int64_t, double, double, GemmEpi, double*, double*, hipStream_t);
template void launch_gemm_tall<bf16>(int64_t, int, int, const bf16*, int64_t, int, const bf16*, int64_t, const float*, int64_t, bf16*, int64_t, double, double, GemmEpi, double*, double*, hipStream_t);

template <typename C>
void launch_cholesky(int l, const double* G, int64_t ldg, double shift, double rel_tol, double* R64,
                     C* Rc, C* Dinv_c, int* flag, int retry, hipStream_t stream) {
  const int T = pad16(l) / 16;
  const size_t lds = T <= kCholLdsMaxTiles ? static_cast<size_t>(T) * (T + 1) / 2 * 256 * sizeof(double) : 0;
  if (T <= kCholLdsMaxTiles)
    hipLaunchKernelGGL((cholesky_kernel<C, true>), dim3(1), dim3(kCholThreads), lds, stream, l, G, ldg, shift,
                       rel_tol, R64, Rc, Dinv_c, flag, retry);
  else
    hipLaunchKernelGGL((cholesky_kernel<C, false>), dim3(1), dim3(kCholThreads), 0, stream, l, G, ldg, shift,
                       rel_tol, R64, Rc, Dinv_c, flag, retry);
  ISVD_LAUNCH_CHECK();
}
template void launch_cholesky<double>(int, const double*, int64_t, double, double, double*, double*, double*, int*, int, hipStream_t);
template void launch_cholesky<float>(int, const double*, int64_t, double, double, double*, float*, float*, int*, int, hipStream_t);

template <typename T>
void launch_trsm_tall(int64_t rows, int l, T* Y, int64_t ld, const typename ComputeOf<T>::type* Rc,
                      const typename ComputeOf<T>::type* Dinv, double* colsum, double* work,
                      hipStream_t stream) {
  using C = typename ComputeOf<T>::type;
  if (rows <= 0) return;
  auto lds_for = [&](int w) {
    return (static_cast<size_t>(w) * 16 * (pad16(l) + 1) + static_cast<size_t>(pad16(l)) * 16 + 256) * sizeof(C) +
           (static_cast<size_t>(pad16(l)) + 64) * sizeof(double);
  };
  int waves = sizeof(C) == 8 ? 2 : 4;
  while (waves > 1 && lds_for(waves) > 160 * 1024) waves /= 2;
  const size_t lds = lds_for(waves);
  ISVD_CHECK(lds <= 160 * 1024, ISVD_E_INVALID, "trsm: block too wide");
  const int64_t nblk = ceil_div(rows, 16 * waves);
  const int64_t grid = colsum ? (nblk < kTrsmParts ? nblk : kTrsmParts) : nblk;
  hipLaunchKernelGGL((trsm_tall_kernel<T, C>), dim3(static_cast<unsigned>(grid)), dim3(64 * waves), lds, stream,
                     rows, l, Y, ld, Rc, Dinv, colsum ? work : nullptr);
  ISVD_LAUNCH_CHECK();
  if (colsum) {
    hipLaunchKernelGGL(colpart_reduce_kernel, dim3(l), dim3(256), 0, stream, static_cast<int>(grid), l, work, colsum);
    ISVD_LAUNCH_CHECK();
  }
}
template void launch_trsm_tall<double>(int64_t, int, double*, int64_t, const double*, const double*, double*, double*, hipStream_t);
template void launch_trsm_tall<float>(int64_t, int, float*, int64_t, const float*, const float*, double*, double*, hipStream_t);
template void launch_trsm_tall<bf16>(int64_t, int, bf16*, int64_t, const float*, const float*, double*, double*, hipStream_t);

int trsm_rows_max_l(int esize) { return esize == 8 ? 128 : 320; }

size_t trsm_rows_packed_elems(int l) {
  const int TT = pad16(l) / 16;
  return static_cast<size_t>(TT) * (TT + 1) / 2 * 256;
}

template <typename C>
void launch_trsm_rows_pack(int l, const double* R64, const double* Dinv64, C* Rf, hipStream_t stream) {
  const int lp = pad16(l);
  const int64_t total = static_cast<int64_t>(trsm_rows_packed_elems(l));
  hipLaunchKernelGGL((rfrag_pack_kernel<C>), dim3(static_cast<unsigned>(ceil_div(total, 256))), dim3(256), 0, stream,
                     lp, R64, Dinv64, Rf);
  ISVD_LAUNCH_CHECK();
}
template void launch_trsm_rows_pack<double>(int, const double*, const double*, double*, hipStream_t);
template void launch_trsm_rows_pack<float>(int, const double*, const double*, float*, hipStream_t);

constexpr size_t kTrsmRowsMaxLds = 96 * 1024;
constexpr int kTrsmWideWaves = 8;

// LDS bytes a workgroup may use on the current device (cached per device).
size_t lds_per_block() {
  static std::mutex mu;
  static std::map<int, size_t> cache;
  int dev = 0;
  ISVD_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int v = 0;
  ISVD_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  cache.emplace(dev, static_cast<size_t>(v > 0 ? v : 0));
  return static_cast<size_t>(v > 0 ? v : 0);
}

// Workgroups of `fn` (threads, dynamic LDS bytes) the current device holds at
// once; cached per (kernel, LDS, device).
int resident_workgroups(const void* fn, int threads, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, size_t, int>, int> cache;
  int dev = 0;
  ISVD_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_tuple(fn, lds, dev);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  ISVD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds));
  ISVD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int n = std::max(1, per_cu) * std::max(1, cus);
  cache.emplace(key, n);
  return n;
}

// The grid-stride row loop runs in one round of resident workgroups (a
// partial second round would leave most of the chip idle at the end).
// Returns the grid launched (the number of column-sum partials written).
template <typename T, typename C, int MT>
int64_t trsm_rows_launch(int64_t rows, int l, T* Y, int64_t ld, int vec, const C* Rf, double* colpart, int64_t grid,
                      hipStream_t stream) {
  if constexpr (MT <= 12) {
    const size_t packed = trsm_rows_packed_elems(l) * sizeof(C);
    const bool staged = packed <= kTrsmRowsMaxLds;
    const void* fn = staged ? reinterpret_cast<const void*>(&trsm_rows_kernel<T, C, MT, true>)
                            : reinterpret_cast<const void*>(&trsm_rows_kernel<T, C, MT, false>);
    const int64_t resident = resident_workgroups(fn, 256, staged ? packed : 0);
    if (grid > resident) grid = resident;
    if (staged)
      hipLaunchKernelGGL((trsm_rows_kernel<T, C, MT, true>), dim3(static_cast<unsigned>(grid)), dim3(256), packed,
                         stream, rows, l, Y, ld, vec, Rf, colpart);
    else
      hipLaunchKernelGGL((trsm_rows_kernel<T, C, MT, false>), dim3(static_cast<unsigned>(grid)), dim3(256), 0,
                         stream, rows, l, Y, ld, vec, Rf, colpart);
  } else {
    if constexpr (std::is_same<C, float>::value && (MT == 16 || MT == 18)) {
      // whole tiles, aligned rows: the off-diagonal tiles in the LDS of one workgroup per CU
      const size_t lds = static_cast<size_t>(MT) * (MT - 1) / 2 * 256 * sizeof(float);
      const size_t sums = static_cast<size_t>(kTrsmWideWaves) * 16 * MT * sizeof(double);
      const size_t need = lds > sums ? lds : sums;
      if (l == 16 * MT && vec && need <= lds_per_block()) {
        const void* fn = reinterpret_cast<const void*>(&trsm_wide_kernel<T, MT, kTrsmWideWaves>);
        const int64_t resident = resident_workgroups(fn, 64 * kTrsmWideWaves, need);
        const int64_t want = ceil_div(ceil_div(rows, 16), kTrsmWideWaves);
        grid = std::min<int64_t>(std::min<int64_t>(resident, want), kRowsTrsmParts);
        hipLaunchKernelGGL((trsm_wide_kernel<T, MT, kTrsmWideWaves>), dim3(static_cast<unsigned>(grid)),
                           dim3(64 * kTrsmWideWaves), need, stream, rows, Y, ld, Rf, colpart);
        ISVD_LAUNCH_CHECK();
        return grid;
      }
    }
    // the factor is read from global memory (it does not fit in LDS)
    const int64_t resident =
        resident_workgroups(reinterpret_cast<const void*>(&trsm_rows_kernel<T, C, MT, false>), 256, 0);
    if (grid > resident) grid = resident;
    hipLaunchKernelGGL((trsm_rows_kernel<T, C, MT, false>), dim3(static_cast<unsigned>(grid)), dim3(256), 0,
                       stream, rows, l, Y, ld, vec, Rf, colpart);
  }
  ISVD_LAUNCH_CHECK();
  return grid;
}

template <typename T>
void launch_trsm_rows(int64_t rows, int l, T* Y, int64_t ld, const typename ComputeOf<T>::type* Rf, double* colsum,
                      double* work, hipStream_t stream) {
  using C = typename ComputeOf<T>::type;
  ISVD_CHECK(l >= 1 && l <= trsm_rows_max_l(static_cast<int>(sizeof(C))), ISVD_E_INVALID,
             "row-register triangular solve: l out of range");
  if (rows <= 0) {
    if (colsum) {
      hipLaunchKernelGGL(zero_doubles_kernel, dim3(static_cast<unsigned>(ceil_div(l, 256))), dim3(256), 0, stream,
                         static_cast<int64_t>(l), colsum);
      ISVD_LAUNCH_CHECK();
    }
    return;
  }
  const int vec = (ld % 4 == 0 && (reinterpret_cast<uintptr_t>(Y) % (4 * sizeof(T))) == 0) ? 1 : 0;
  const int64_t ntiles = ceil_div(rows, 16);
  const int64_t want = ceil_div(ntiles, 4);
  int64_t grid = want < kRowsTrsmParts ? want : kRowsTrsmParts;
  double* part = colsum ? work : nullptr;
  const int TT = pad16(l) / 16;
  if constexpr (sizeof(C) == 8) {
    if (TT <= 4) grid = trsm_rows_launch<T, C, 4>(rows, l, Y, ld, vec, Rf, part, grid, stream);
    else grid = trsm_rows_launch<T, C, 8>(rows, l, Y, ld, vec, Rf, part, grid, stream);
  } else {
    if (TT <= 4) grid = trsm_rows_launch<T, C, 4>(rows, l, Y, ld, vec, Rf, part, grid, stream);
    else if (TT <= 8) grid = trsm_rows_launch<T, C, 8>(rows, l, Y, ld, vec, Rf, part, grid, stream);
    else if (TT <= 9) grid = trsm_rows_launch<T, C, 9>(rows, l, Y, ld, vec, Rf, part, grid, stream);
    else if (TT <= 12) grid = trsm_rows_launch<T, C, 12>(rows, l, Y, ld, vec, Rf, part, grid, stream);
    else if (TT <= 16) grid = trsm_rows_launch<T, C, 16>(rows, l, Y, ld, vec, Rf, part, grid, stream);
    else if (TT <= 18) grid = trsm_rows_launch<T, C, 18>(rows, l, Y, ld, vec, Rf, part, grid, stream);
    else grid = trsm_rows_launch<T, C, 20>(rows, l, Y, ld, vec, Rf, part, grid, stream);
  }
  if (colsum) {
    hipLaunchKernelGGL(colpart_reduce_kernel, dim3(l), dim3(256), 0, stream, static_cast<int>(grid), l, work, colsum);
    ISVD_LAUNCH_CHECK();
  }
}
template void launch_trsm_rows<double>(int64_t, int, double*, int64_t, const double*, double*, double*, hipStream_t);
template void launch_trsm_rows<float>(int64_t, int, float*, int64_t, const float*, double*, double*, hipStream_t);
template void launch_trsm_rows<bf16>(int64_t, int, bf16*, int64_t, const float*, double*, double*, hipStream_t);

void launch_upper_mult(int l, const double* A, const double* B, double* Cm, int64_t ld, hipStream_t stream) {
  const int lp = pad16(l);
  const int64_t total = static_cast<int64_t>(lp) * lp;
  hipLaunchKernelGGL(upper_mult_kernel, dim3(static_cast<unsigned>(ceil_div(total, 256))), dim3(256), 0,
                     stream, lp, A, B, Cm, ld);
  ISVD_LAUNCH_CHECK();
}

size_t jacobi_workspace_doubles(int n) {
  const int np = static_cast<int>(round_up(n, 32));  // covers the padding of both variants
  return 2 * static_cast<size_t>(np) * n + 2 * static_cast<size_t>(np) + 96;
}

void launch_jacobi_svd(int n, const double* A, int64_t lda, double* U, double* s, double* V, double* work,
                       int* sweeps_out, hipStream_t stream, const double* V0, double rel_tol) {
  ISVD_CHECK(n >= 1 && n <= kJacobiMaxN, ISVD_E_INVALID, "small svd: n out of range");
  if (n <= 64 || n > 512) {
    // one workgroup, pairs held in registers
    if (n <= 8 * kJacobiPerLane)
      hipLaunchKernelGGL(jacobi_kernel<8>, dim3(1), dim3(1024), 0, stream, n, A, lda, U, s, V, work, sweeps_out);
    else if (n <= 16 * kJacobiPerLane)
      hipLaunchKernelGGL(jacobi_kernel<16>, dim3(1), dim3(1024), 0, stream, n, A, lda, U, s, V, work, sweeps_out);
    else if (n <= 32 * kJacobiPerLane)
      hipLaunchKernelGGL(jacobi_kernel<32>, dim3(1), dim3(1024), 0, stream, n, A, lda, U, s, V, work, sweeps_out);
    else
      hipLaunchKernelGGL(jacobi_kernel<64>, dim3(1), dim3(1024), 0, stream, n, A, lda, U, s, V, work, sweeps_out);
    ISVD_LAUNCH_CHECK();
    return;
  }
  // block-parallel version: blocks of B columns, an even number of blocks
  const int B = n <= 304 ? 16 : 8;
  int nbk = static_cast<int>(ceil_div(n, B));
  nbk += nbk & 1;
  const int np = nbk * B;
  double* Wt = work;
  double* Jt = Wt + static_cast<int64_t>(np) * n;
  double* sig = Jt + static_cast<int64_t>(np) * n;
  int* rank = reinterpret_cast<int*>(sig + n);
  int* flags = rank + n + 1;
  const int nflags = 1 + 64 + 2;
  const int64_t total = static_cast<int64_t>(np) * n;
  hipLaunchKernelGGL(bjacobi_init_kernel, dim3(static_cast<unsigned>(ceil_div(total, 256))), dim3(256), 0, stream, n, np,
                     A, lda, V0, Wt, Jt, flags, nflags);
  ISVD_LAUNCH_CHECK();
  const int per = static_cast<int>(ceil_div(n, 16));
  auto round_launch = [&](int r, int sweep) {
    const dim3 grid(nbk / 2), block(16 * B);
    // 2B columns of W and of J, stride 16 PER (PER: the template argument)
    auto lds_of = [&](int PER) { return static_cast<size_t>(4) * B * 16 * PER * sizeof(double); };
    if (B == 16) {
      if (per <= 5)
        hipLaunchKernelGGL((bjacobi_round_kernel<16, 5>), grid, block, lds_of(5), stream, n, nbk, r, sweep, Wt, Jt, flags, rel_tol);
      else if (per <= 9)
        hipLaunchKernelGGL((bjacobi_round_kernel<16, 9>), grid, block, lds_of(9), stream, n, nbk, r, sweep, Wt, Jt, flags, rel_tol);
      else if (per <= 13)
        hipLaunchKernelGGL((bjacobi_round_kernel<16, 13>), grid, block, lds_of(13), stream, n, nbk, r, sweep, Wt, Jt, flags, rel_tol);
      else
        hipLaunchKernelGGL((bjacobi_round_kernel<16, 19>), grid, block, lds_of(19), stream, n, nbk, r, sweep, Wt, Jt, flags, rel_tol);
    } else {
      if (per <= 26)
        hipLaunchKernelGGL((bjacobi_round_kernel<8, 26>), grid, block, lds_of(26), stream, n, nbk, r, sweep, Wt, Jt, flags, rel_tol);
      else
        hipLaunchKernelGGL((bjacobi_round_kernel<8, 32>), grid, block, lds_of(32), stream, n, nbk, r, sweep, Wt, Jt, flags, rel_tol);
    }
  };
  constexpr int kMaxSweeps = 40;
  int done = 0;
  for (int sweep = 0; sweep < kMaxSweeps && !done; ++sweep) {
    for (int r = 0; r < nbk - 1; ++r) round_launch(r, sweep);
    hipLaunchKernelGGL(bjacobi_check_kernel, dim3(1), dim3(64), 0, stream, sweep, flags);
    ISVD_LAUNCH_CHECK();
    // read the convergence flag after every sweep from the third on (a sweep
    // costs far more than the host round trip)
    if (sweep >= 2) {
      ISVD_HIP(hipMemcpyAsync(&done, flags, sizeof(int), hipMemcpyDeviceToHost, stream));
      ISVD_HIP(hipStreamSynchronize(stream));
    }
  }
  hipLaunchKernelGGL(bjacobi_finish_kernel, dim3(1), dim3(1024), 0, stream, n, Wt, Jt, U, s, V, sig, rank, flags,
                     sweeps_out);
  ISVD_LAUNCH_CHECK();
}

template <typename T>
void launch_gaussian(int64_t rows, int64_t cols, uint64_t seed, T* out, int64_t ld, hipStream_t stream) {
  const int64_t pairs = ceil_div(rows * cols, 2);
  if (pairs == 0) return;
  hipLaunchKernelGGL(gaussian_kernel<T>, dim3(static_cast<unsigned>(ceil_div(pairs, 256))), dim3(256), 0,
                     stream, rows, cols, seed, out, ld);
  ISVD_LAUNCH_CHECK();
}
template void launch_gaussian<double>(int64_t, int64_t, uint64_t, double*, int64_t, hipStream_t);
template void launch_gaussian<float>(int64_t, int64_t, uint64_t, float*, int64_t, hipStream_t);
template void launch_gaussian<bf16>(int64_t, int64_t, uint64_t, bf16*, int64_t, hipStream_t);

template <typename D, typename S>
void launch_convert(int64_t rows, int64_t cols, const S* src, int64_t lds, D* dst, int64_t ldd,
                    hipStream_t stream) {
  const int64_t total = rows * cols;
  if (total == 0) return;
  hipLaunchKernelGGL((convert_kernel<D, S>), dim3(static_cast<unsigned>(ceil_div(total, 256))), dim3(256),
                     0, stream, rows, cols, src, lds, dst, ldd);
  ISVD_LAUNCH_CHECK();
}
template void launch_convert<float, bf16>(int64_t, int64_t, const bf16*, int64_t, float*, int64_t, hipStream_t);
template void launch_convert<bf16, float>(int64_t, int64_t, const float*, int64_t, bf16*, int64_t, hipStream_t);
template void launch_convert<float, float>(int64_t, int64_t, const float*, int64_t, float*, int64_t, hipStream_t);
template void launch_convert<double, double>(int64_t, int64_t, const double*, int64_t, double*, int64_t, hipStream_t);
template void launch_convert<bf16, bf16>(int64_t, int64_t, const bf16*, int64_t, bf16*, int64_t, hipStream_t);
template void launch_convert<float, double>(int64_t, int64_t, const double*, int64_t, float*, int64_t, hipStream_t);
template void launch_convert<double, float>(int64_t, int64_t, const float*, int64_t, double*, int64_t, hipStream_t);

template <typename C>
void launch_pack_residual_rhs(int l, int k, const double* UR, const double* ZR, const double* s, int64_t ld,
                              C* B, hipStream_t stream) {
  hipLaunchKernelGGL((pack_residual_rhs_kernel<C>), dim3(static_cast<unsigned>(ceil_div(2 * l * k, 256))),
                     dim3(256), 0, stream, l, k, UR, ZR, s, ld, B);
  ISVD_LAUNCH_CHECK();
}
template void launch_pack_residual_rhs<float>(int, int, const double*, const double*, const double*, int64_t, float*, hipStream_t);
template void launch_pack_residual_rhs<double>(int, int, const double*, const double*, const double*, int64_t, double*, hipStream_t);

void launch_small_residual(int l, int k, const double* Rc, int64_t ldr, const double* ZR, const double* UR,
                           int64_t ldu, const double* s, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(small_residual_kernel, dim3(k), dim3(256), 0, stream, l, k, Rc, ldr, ZR, UR, ldu, s, out);
  ISVD_LAUNCH_CHECK();
}

}  // namespace isvd
