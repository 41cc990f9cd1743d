#pragma once

#include "common.h"

namespace hicu {

int32_t launch_jl(const float2* Q, int n, int nq, int p, uint64_t seed, uint32_t outer, uint32_t inner,
                  uint32_t sid, float2* F, double* Pout, hipStream_t st);
// Randomized-SVD sketch Omega (n x l complex64) for (seed, outer, sid).
int32_t launch_sketch(int n, int ell, uint64_t seed, uint32_t outer, uint32_t sid, float2* Om, hipStream_t st);
int32_t launch_eta(const double* part, int64_t count, const double* gnorm2, double* eta, hipStream_t st);
int32_t launch_update(float2* x, const float2* g, const double* eta, int64_t count, hipStream_t st);
int32_t launch_zero(void* ptr, size_t bytes, hipStream_t st);
struct KMaskBits {
  uint64_t w[8];
};
// Spread filters over a kernel mask's taps (g.n rows) to the whole box
// (g.nbox rows, zero outside the mask).
int32_t launch_kmask_scatter(const Geo& g, const float2* F, int p, float2* Fbox, hipStream_t st);
// Time-averaged initialisation along canonical axis `axis` of extents d.
int32_t launch_time_average(const float2* x0, const uint8_t* mask, float2* out, const int64_t d[3], int axis,
                            int nc, hipStream_t st);
// *out = number of non-finite values among the `count` floats at v.
int32_t launch_count_nonfinite(const float* v, int64_t count, unsigned long long* out, hipStream_t st);

// FP16 operand scaling.  launch_absmax writes per-block maxima of |v| over
// `count` floats into part (kAbsmaxBlocks entries); launch_scale turns
// `count` maxima into the power of two 2^(14 - ceil(log2 max)) (1 for a
// zero or non-finite maximum) at *scale.
constexpr int kAbsmaxBlocks = 512;
int32_t launch_absmax(const float* v, int64_t count, float* part, hipStream_t st);
int32_t launch_scale(const float* part, int64_t count, float* scale, hipStream_t st);

}  // namespace hicu
