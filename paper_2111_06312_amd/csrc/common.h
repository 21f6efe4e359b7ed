// Shared device/host helpers for the implicit-SVD library (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstdio>
#include <string>

#include "isvd.h"

namespace isvd {

// ---------------------------------------------------------------- errors

void set_last_error(const std::string& msg);

struct Error {
  isvd_status code;
  std::string msg;
};

#define ISVD_HIP(expr)                                                              \
  do {                                                                              \
    hipError_t _e = (expr);                                                         \
    if (_e != hipSuccess) {                                                         \
      throw ::isvd::Error{_e == hipErrorOutOfMemory ? ISVD_E_OOM : ISVD_E_HIP,      \
                          std::string(#expr) + ": " + hipGetErrorString(_e)};       \
    }                                                                               \
  } while (0)

#define ISVD_CHECK(cond, code, msg)                                                 \
  do {                                                                              \
    if (!(cond)) throw ::isvd::Error{code, msg};                                    \
  } while (0)

#define ISVD_LAUNCH_CHECK() ISVD_HIP(hipGetLastError())

// ---------------------------------------------------------------- bf16

// Brain float stored as its 16-bit pattern.
struct bf16 {
  uint16_t bits;
};

__host__ __device__ inline float bf16_to_float(uint16_t b) {
  union { uint32_t u; float f; } v;
  v.u = static_cast<uint32_t>(b) << 16;
  return v.f;
}

// Round to nearest, ties to even, on the bits and without branches; NaN
// stays NaN (quiet).  (The packed conversion instruction of gfx950 was
// measured to round ties to the odd neighbour.)
__host__ __device__ inline uint32_t bf16_round_high(float f) {
  union { uint32_t u; float f; } v;
  v.f = f;
  const uint32_t u = v.u;
  const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return (u & 0x7fffffffu) > 0x7f800000u ? (u | 0x400000u) : r;   // the result in bits 31..16
}
__host__ __device__ inline uint16_t float_to_bf16(float f) { return static_cast<uint16_t>(bf16_round_high(f) >> 16); }
__host__ __device__ inline uint32_t float2_to_bf16x2(float lo, float hi) {
  return (bf16_round_high(lo) >> 16) | (bf16_round_high(hi) & 0xffff0000u);
}

// Element conversions between storage types and compute types.
template <typename T> struct Elem;
template <> struct Elem<double> {
  __device__ static inline double load(const double* p) { return *p; }
  __device__ static inline void store(double* p, double v) { *p = v; }
  __device__ static inline double to_d(double v) { return v; }
};
template <> struct Elem<float> {
  __device__ static inline float load(const float* p) { return *p; }
  __device__ static inline void store(float* p, float v) { *p = v; }
};
template <> struct Elem<bf16> {
  __device__ static inline float load(const bf16* p) { return bf16_to_float(p->bits); }
  __device__ static inline void store(bf16* p, float v) { p->bits = float_to_bf16(v); }
};

// Compute type used for a storage type: FP64 stays FP64, FP32 and BF16 compute in FP32.
template <typename T> struct ComputeOf { using type = float; };
template <> struct ComputeOf<double> { using type = double; };

template <typename A, typename B>
__device__ inline A cvt(B v) { return static_cast<A>(v); }

inline size_t elem_size(isvd_precision p) {
  return p == ISVD_FP64 ? 8 : (p == ISVD_FP32 ? 4 : 2);
}

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
inline int64_t ceil_div(int64_t x, int64_t m) { return (x + m - 1) / m; }

// ---------------------------------------------------------------- wave helpers

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline float wave_sum(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Lane exchange within each row of 16 lanes through a DPP operand (no LDS
// round trip).  Every lane of the wave must be active.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of a row, returned to all of them: swap neighbours,
// then pairs, then quads (half-row mirror), then halves (row mirror).  Each
// step adds the same two operands on both partner lanes, so every lane of the
// row ends with the same bits.
__device__ inline double row16_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return v;
}

// Four sums over the 16 lanes of a row at once (a reduce-scatter): lane li
// returns the row's sum of v[row16_sum4_index(li)].  Neighbours, then pairs,
// exchange half of what they hold; the four quads are then added by
// rotations of 4 and 8 lanes, which keep li mod 4.  Lanes that return the
// same index may differ in the last bits (the additions are associated
// differently); callers take each sum from a fixed lane.
__device__ inline int row16_sum4_index(int li) { return 2 * (li & 1) + ((li >> 1) & 1); }
__device__ inline double row16_sum4(const double (&v)[4], int li) {
  const bool odd = (li & 1) != 0;
  double k0 = odd ? v[2] : v[0], k1 = odd ? v[3] : v[1];
  const double s0 = odd ? v[0] : v[2], s1 = odd ? v[1] : v[3];
  k0 += dpp_f64<0xB1>(s0);   // quad_perm [1,0,3,2]
  k1 += dpp_f64<0xB1>(s1);
  const bool hi = (li & 2) != 0;
  double k = hi ? k1 : k0;
  const double s = hi ? k0 : k1;
  k += dpp_f64<0x4E>(s);     // quad_perm [2,3,0,1]
  k += dpp_f64<0x124>(k);    // row_ror:4
  k += dpp_f64<0x128>(k);    // row_ror:8
  return k;
}

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- device buffers

// Owning device allocation (hipMalloc / hipFree).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t n) {
    if (n <= bytes) return;
    release();
    ISVD_HIP(hipMalloc(&p, n));
    bytes = n;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

}  // namespace isvd
