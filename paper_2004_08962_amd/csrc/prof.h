// Optional per-kernel timing with HIP events recorded on the launch stream.
#pragma once

#include "common.h"

namespace hicu {

bool prof_on();

// While an object of this type is alive, ProfScope records nothing on the
// calling thread (for entry points that must not create events).
class ProfSuppress {
 public:
  ProfSuppress();
  ~ProfSuppress();
  ProfSuppress(const ProfSuppress&) = delete;
  ProfSuppress& operator=(const ProfSuppress&) = delete;
};

// Records a start event at construction and a stop event at destruction on
// `st` when profiling is enabled; `flops`/`bytes` are the algorithmic work of
// the bracketed launch.  `minor` marks the per-step scalar and layout
// kernels, which a major-only profile leaves untimed.
class ProfScope {
 public:
  ProfScope(const char* tag, hipStream_t st, double flops = 0.0, double bytes = 0.0, bool minor = false);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  const char* tag_;
  hipStream_t st_;
  double flops_, bytes_;
  hipEvent_t a_ = nullptr;
};

}  // namespace hicu
