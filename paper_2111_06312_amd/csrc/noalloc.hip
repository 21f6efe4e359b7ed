// The Gram product A^T B for callers that cannot allocate device memory
// (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc): its row-slice partial results live in one fixed array of this
// library instead of a workspace allocated per call.
//
// The array is a file-scope __device__ variable: every GPU the library runs
// on holds its own copy, at its own address, until the process ends.  In host
// code the array's name is not a device address, so its address is taken
// once per device with hipGetSymbolAddress (with that device current) and
// only that pointer is handed to kernels.  Every call on a GPU shares the
// array: calls that overlap in time on one GPU (different streams, or other
// threads) race on it and must be serialised by the caller.  The partial
// tiles a call reads are all written earlier in the same call, so nothing
// needs clearing between calls.
#include <mutex>

#include "dense.h"

namespace isvd {

namespace {

constexpr size_t kScratchDoubles = static_cast<size_t>(32) << 17;   // 32 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

size_t scratch_doubles() { return kScratchDoubles; }

// Device address of the current device's copy of `scratch` (looked up once
// per device).
double* scratch_ptr() {
  int dev = 0;
  ISVD_HIP(hipGetDevice(&dev));
  ISVD_CHECK(dev >= 0 && dev < kMaxDevices, ISVD_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    ISVD_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    ISVD_CHECK(ptr != nullptr, ISVD_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[dev];
}

template <typename T>
void gram_noalloc(int64_t rows, int m, int p, const T* A, int64_t lda, const T* B, int64_t ldb, bool same, double* C,
                  int64_t ldc, hipStream_t stream) {
  launch_gram_bounded<T>(rows, m, p, A, lda, B, ldb, same, C, ldc, scratch_ptr(), kScratchDoubles, stream);
}
template void gram_noalloc<double>(int64_t, int, int, const double*, int64_t, const double*, int64_t, bool, double*, int64_t, hipStream_t);
template void gram_noalloc<float>(int64_t, int, int, const float*, int64_t, const float*, int64_t, bool, double*, int64_t, hipStream_t);
template void gram_noalloc<bf16>(int64_t, int, int, const bf16*, int64_t, const bf16*, int64_t, bool, double*, int64_t, hipStream_t);

}  // namespace isvd
