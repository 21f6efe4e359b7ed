// Opt-in per-launch timing: a start/stop hipEvent pair on the launch stream
// around every timed region, plus its algorithmic byte counts.  Class 0 is
// the sparse pass; classes 1..3 are the learner kernels (embeddings, pair
// scores, the least-norm model chain).
#include <mutex>
#include <vector>

#include "spmm.h"

namespace isvd {

namespace {
struct Rec {
  hipEvent_t a = nullptr, b = nullptr;
  double bytes = 0.0, bytes2 = 0.0;
  int tag = 0;   // sparse passes: bytes per block element
};
struct Pool {
  std::vector<Rec> recs;
  size_t used = 0;
};
std::mutex g_mu;
bool g_on = false;
Pool g_pools[kProfileClasses];
}  // namespace

bool spmm_profiling() { return g_on; }

void* profile_begin(int cls, hipStream_t stream, double bytes, double bytes2, int tag) {
  std::lock_guard<std::mutex> lk(g_mu);
  Pool& p = g_pools[cls];
  if (p.used == p.recs.size()) {
    Rec r;
    ISVD_HIP(hipEventCreate(&r.a));
    ISVD_HIP(hipEventCreate(&r.b));
    p.recs.push_back(r);
  }
  Rec& r = p.recs[p.used];
  r.bytes = bytes;
  r.bytes2 = bytes2;
  r.tag = tag;
  ISVD_HIP(hipEventRecord(r.a, stream));
  // token = class and index + 1 (never null)
  return reinterpret_cast<void*>((static_cast<size_t>(cls) << 48) | ++p.used);
}

void profile_end(hipStream_t stream, void* token) {
  std::lock_guard<std::mutex> lk(g_mu);
  const size_t t = reinterpret_cast<size_t>(token);
  ISVD_HIP(hipEventRecord(g_pools[t >> 48].recs[(t & ((size_t(1) << 48) - 1)) - 1].b, stream));
}

void* spmm_profile_begin(hipStream_t stream, double gather_bytes, double compulsory_bytes, int elem_bytes) {
  return profile_begin(0, stream, gather_bytes, compulsory_bytes, elem_bytes);
}

void spmm_profile_end(hipStream_t stream, void* token) { profile_end(stream, token); }

void spmm_profile_enable(bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on;
  for (Pool& p : g_pools) p.used = 0;
}

void profile_read(int cls, double* ms, double* bytes, double* bytes2, int64_t* launches, int tag, bool clear) {
  std::lock_guard<std::mutex> lk(g_mu);
  Pool& p = g_pools[cls];
  double t = 0.0, b = 0.0, b2 = 0.0;
  int64_t n = 0;
  for (size_t i = 0; i < p.used; ++i) {
    if (tag && p.recs[i].tag != tag) continue;
    ++n;
    ISVD_HIP(hipEventSynchronize(p.recs[i].b));
    float e = 0.f;
    ISVD_HIP(hipEventElapsedTime(&e, p.recs[i].a, p.recs[i].b));
    t += e;
    b += p.recs[i].bytes;
    b2 += p.recs[i].bytes2;
  }
  *ms = t;
  *bytes = b;
  if (bytes2) *bytes2 = b2;
  *launches = n;
  if (clear) p.used = 0;
}

void spmm_profile_read(double* ms, double* gather, double* compulsory, int64_t* launches, int elem_bytes,
                       bool clear) {
  profile_read(0, ms, gather, compulsory, launches, elem_bytes, clear);
}

}  // namespace isvd
