// Peak rates of the device, measured for the rooflines of the library's
// kernels: a streaming copy (HBM), repeated reads of a buffer that fits the
// Infinity Cache but not the L2s, and back-to-back independent MFMAs (FP64
// and FP32 16x16x4).  Each entry point times its launches with a hipEvent
// pair on the given stream and waits for them.
#include "common.h"

namespace isvd {

namespace {

constexpr int kPeakThreads = 256;

__global__ __launch_bounds__(kPeakThreads) void peak_copy_kernel(const uint4* src, uint4* dst, int64_t n16) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  // four 16-byte loads in flight per thread before their stores
  for (; i + 3 * stride < n16; i += 4 * stride) {
    uint4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u) dst[i + u * stride] = v[u];
  }
  for (; i < n16; i += stride) dst[i] = src[i];
}

// Pass r reads the buffer starting at chunk r * rot (mod n16), so a thread
// meets different lines on every pass (no L2 reuse across passes).
__global__ __launch_bounds__(kPeakThreads) void peak_read_kernel(const uint4* src, int64_t n16, int reps,
                                                                 int64_t rot, uint32_t* sink) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (int r = 0; r < reps; ++r) {
    const int64_t off = (static_cast<int64_t>(r) * rot) % n16;
    int64_t i = t;
    for (; i + 3 * stride < n16; i += 4 * stride) {
      uint4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        int64_t j = i + u * stride + off;
        j = j >= n16 ? j - n16 : j;
        v[u] = src[j];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < n16; i += stride) {
      int64_t j = i + off;
      j = j >= n16 ? j - n16 : j;
      const uint4 v = src[j];
      acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
  }
  sink[t] = acc;
}

typedef double v4d_peak __attribute__((ext_vector_type(4)));
typedef float v4f_peak __attribute__((ext_vector_type(4)));
constexpr int kPeakChains = 8;   // independent accumulators per wave
constexpr int kPeakUnroll = 32;  // MFMA rounds per loop trip: the accumulators move between register files once per trip

__global__ __launch_bounds__(kPeakThreads) void peak_mfma_f64_kernel(int64_t iters, double* sink) {
  v4d_peak acc[kPeakChains];
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) acc[c] = v4d_peak{0.0, 0.0, 0.0, 0.0};
  const double a = 1.0 + 1e-9 * threadIdx.x, b = 1.0 - 1e-9 * threadIdx.x;
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kPeakUnroll; ++u)
#pragma unroll
      for (int c = 0; c < kPeakChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  sink[static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(kPeakThreads) void peak_mfma_f32_kernel(int64_t iters, double* sink) {
  v4f_peak acc[kPeakChains];
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) acc[c] = v4f_peak{0.f, 0.f, 0.f, 0.f};
  const float a = 1.0f + 1e-6f * threadIdx.x, b = 1.0f - 1e-6f * threadIdx.x;
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kPeakUnroll; ++u)
#pragma unroll
      for (int c = 0; c < kPeakChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  sink[static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    ISVD_HIP(hipEventCreate(&a));
    ISVD_HIP(hipEventCreate(&b));
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  double wait_ms() {
    ISVD_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    ISVD_HIP(hipEventElapsedTime(&ms, a, b));
    return ms;
  }
};

int device_cus() {
  int dev = 0, cus = 0;
  ISVD_HIP(hipGetDevice(&dev));
  ISVD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  return cus > 0 ? cus : 1;
}

}  // namespace

double peak_copy(const void* src, void* dst, int64_t bytes, int reps, hipStream_t stream) {
  const int64_t n16 = bytes / 16;
  const unsigned grid = static_cast<unsigned>(device_cus() * 16);
  EventPair ev;
  ISVD_HIP(hipEventRecord(ev.a, stream));
  for (int r = 0; r < reps; ++r) {
    hipLaunchKernelGGL(peak_copy_kernel, dim3(grid), dim3(kPeakThreads), 0, stream, static_cast<const uint4*>(src),
                       static_cast<uint4*>(dst), n16);
    ISVD_LAUNCH_CHECK();
  }
  ISVD_HIP(hipEventRecord(ev.b, stream));
  return ev.wait_ms();
}

double peak_read(const void* src, int64_t bytes, int reps, uint32_t* sink, hipStream_t stream) {
  const int64_t n16 = bytes / 16;
  const unsigned grid = static_cast<unsigned>(device_cus() * 16);
  const int64_t rot = n16 / 3 + 1;
  EventPair ev;
  ISVD_HIP(hipEventRecord(ev.a, stream));
  hipLaunchKernelGGL(peak_read_kernel, dim3(grid), dim3(kPeakThreads), 0, stream, static_cast<const uint4*>(src),
                     n16, reps, rot, sink);
  ISVD_LAUNCH_CHECK();
  ISVD_HIP(hipEventRecord(ev.b, stream));
  return ev.wait_ms();
}

int64_t peak_sink_elems() { return static_cast<int64_t>(device_cus()) * 16 * kPeakThreads; }

double peak_mfma(bool fp64, int64_t iters, double* sink, double* flops, hipStream_t stream) {
  const unsigned grid = static_cast<unsigned>(device_cus() * 16);   // 4 waves per block, 16 blocks per CU
  EventPair ev;
  ISVD_HIP(hipEventRecord(ev.a, stream));
  if (fp64)
    hipLaunchKernelGGL(peak_mfma_f64_kernel, dim3(grid), dim3(kPeakThreads), 0, stream, iters, sink);
  else
    hipLaunchKernelGGL(peak_mfma_f32_kernel, dim3(grid), dim3(kPeakThreads), 0, stream, iters, sink);
  ISVD_LAUNCH_CHECK();
  ISVD_HIP(hipEventRecord(ev.b, stream));
  const double waves = static_cast<double>(grid) * (kPeakThreads / 64);
  *flops = waves * static_cast<double>(iters) * kPeakUnroll * kPeakChains * (16.0 * 16.0 * 4.0 * 2.0);
  return ev.wait_ms();
}

}  // namespace isvd
