// Line search with a library-owned scratch buffer, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops,
// harnesses that forbid hipMalloc).  It runs the same kernels as
// hicu_line_search; the workspace (filter weights in fragment order, per-block
// partial sums, FP16 scales) lives in a file-scope device array instead of a
// caller buffer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.h"
#include "prof.h"
#include "step.h"

namespace hicu {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends.  In host code this name is
// only a handle for hipGetSymbolAddress: the kernels receive the device
// address looked up below.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array, looked up once per
// device with that device current.
int32_t scratch_for_current_device(void** out) {
  int dev = -1;
  HICU_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return HICU_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> l(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    HICU_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return HICU_ERR_HIP;
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return HICU_OK;
}

}  // namespace
}  // namespace hicu

using namespace hicu;

extern "C" {

size_t hicu_line_search_noalloc_max_bytes(void) { return kScratchBytes; }

int32_t hicu_line_search_noalloc(const hicu_geom* gm, const void* gv, const double* gn2, const void* F, int32_t p,
                                 int32_t prec, double* eta, void* stream) {
  Geo g;
  HICU_TRY(make_geo(gm, &g));
  if (!gv || !gn2 || !F || !eta || !valid_prec(prec)) return HICU_ERR_ARG;
  if (p < 1 || p > 1 << 20) return HICU_ERR_RANK;
  StepPlan sp;
  HICU_TRY(make_step_plan(g, p, prec, false, &sp));
  if (sp.total > kScratchBytes) return HICU_ERR_WORKSPACE;  // larger than the fixed scratch
  void* ws = nullptr;
  HICU_TRY(scratch_for_current_device(&ws));
  ProfSuppress no_events;  // event timing would create events: not here
  return line_search_impl(g, gv, gn2, F, p, prec, eta, ws, kScratchBytes, (hipStream_t)stream);
}

}  // extern "C"
