// Opt-in per-launch timing of the sparse passes: a start/stop hipEvent pair on
// the launch stream around every pass, plus the pass's algorithmic byte counts.
#include <mutex>
#include <vector>

#include "spmm.h"

namespace isvd {

namespace {
struct Rec {
  hipEvent_t a = nullptr, b = nullptr;
  double gather_bytes = 0.0, compulsory_bytes = 0.0;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_pool;
size_t g_used = 0;
}  // namespace

bool spmm_profiling() { return g_on; }

void* spmm_profile_begin(hipStream_t stream, double gather_bytes, double compulsory_bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_used == g_pool.size()) {
    Rec r;
    ISVD_HIP(hipEventCreate(&r.a));
    ISVD_HIP(hipEventCreate(&r.b));
    g_pool.push_back(r);
  }
  Rec& r = g_pool[g_used];
  r.gather_bytes = gather_bytes;
  r.compulsory_bytes = compulsory_bytes;
  ISVD_HIP(hipEventRecord(r.a, stream));
  return reinterpret_cast<void*>(++g_used);  // token = index + 1 (never null)
}

void spmm_profile_end(hipStream_t stream, void* token) {
  std::lock_guard<std::mutex> lk(g_mu);
  ISVD_HIP(hipEventRecord(g_pool[reinterpret_cast<size_t>(token) - 1].b, stream));
}

void spmm_profile_enable(bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on;
  g_used = 0;
}

void spmm_profile_read(double* ms, double* gather, double* compulsory, int64_t* launches) {
  std::lock_guard<std::mutex> lk(g_mu);
  double t = 0.0, gb = 0.0, cb = 0.0;
  for (size_t i = 0; i < g_used; ++i) {
    ISVD_HIP(hipEventSynchronize(g_pool[i].b));
    float e = 0.f;
    ISVD_HIP(hipEventElapsedTime(&e, g_pool[i].a, g_pool[i].b));
    t += e;
    gb += g_pool[i].gather_bytes;
    cb += g_pool[i].compulsory_bytes;
  }
  *ms = t;
  *gather = gb;
  *compulsory = cb;
  *launches = static_cast<int64_t>(g_used);
  g_used = 0;
}

}  // namespace isvd
