// Per-kernel event timing (see prof.h) and its C ABI.
#include "prof.h"

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace hicu {
namespace {

struct Rec {
  const char* tag;
  hipEvent_t a, b;
  double flops, bytes;
};

std::mutex mu;
bool enabled = false;
bool major_only = false;
thread_local int suppressed = 0;
std::vector<Rec> recs;
std::vector<hipEvent_t> pool;

hipEvent_t get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  // Timing only: no system-scope fence when the event completes (the host
  // reads nothing through these events), which keeps each record cheap.
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

ProfSuppress::ProfSuppress() { ++suppressed; }
ProfSuppress::~ProfSuppress() { --suppressed; }

bool prof_on() {
  std::lock_guard<std::mutex> l(mu);
  return enabled;
}

ProfScope::ProfScope(const char* tag, hipStream_t st, double flops, double bytes, bool minor)
    : tag_(tag), st_(st), flops_(flops), bytes_(bytes) {
  if (suppressed) return;
  std::lock_guard<std::mutex> l(mu);
  if (!enabled || (minor && major_only)) return;
  a_ = get_event();
  if (a_ && hipEventRecord(a_, st_) != hipSuccess) {
    pool.push_back(a_);
    a_ = nullptr;
  }
}

ProfScope::~ProfScope() {
  if (!a_) return;
  std::lock_guard<std::mutex> l(mu);
  hipEvent_t b = get_event();
  if (!b || hipEventRecord(b, st_) != hipSuccess) {
    pool.push_back(a_);
    if (b) pool.push_back(b);
    return;
  }
  recs.push_back(Rec{tag_, a_, b, flops_, bytes_});
}

}  // namespace hicu

using namespace hicu;

extern "C" {

static int32_t profile_start(bool major) {
  std::lock_guard<std::mutex> l(mu);
  for (auto& r : recs) {
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
  enabled = true;
  major_only = major;
  return HICU_OK;
}

int32_t hicu_profile_begin(void) { return profile_start(false); }

int32_t hicu_profile_begin_major(void) { return profile_start(true); }

int32_t hicu_profile_end(hicu_kernel_stat* out, int32_t max_out, int32_t* n_out) {
  std::lock_guard<std::mutex> l(mu);
  enabled = false;
  std::map<std::string, hicu_kernel_stat> acc;
  std::vector<std::string> order;
  int32_t status = HICU_OK;
  for (auto& r : recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      status = HICU_ERR_HIP;
      continue;
    }
    auto it = acc.find(r.tag);
    if (it == acc.end()) {
      hicu_kernel_stat s;
      std::memset(&s, 0, sizeof(s));
      std::strncpy(s.name, r.tag, sizeof(s.name) - 1);
      s.min_ms = 1e300;
      it = acc.emplace(r.tag, s).first;
      order.push_back(r.tag);
    }
    hicu_kernel_stat& s = it->second;
    s.launches += 1;
    s.total_ms += ms;
    s.min_ms = s.min_ms < ms ? s.min_ms : ms;
    s.max_ms = s.max_ms > ms ? s.max_ms : ms;
    s.flops += r.flops;
    s.bytes += r.bytes;
  }
  for (auto& r : recs) {
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
  int32_t n = 0;
  for (const auto& k : order) {
    if (out && n < max_out) out[n] = acc[k];
    ++n;
  }
  if (n_out) *n_out = n;
  return status;
}

}  // extern "C"
