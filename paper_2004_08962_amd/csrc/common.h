// Shared helpers for the HICU HIP library (gfx950 / CDNA4 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "hicu.h"

namespace hicu {

// ---------------------------------------------------------------------------
// Error plumbing (host)
// ---------------------------------------------------------------------------
#define HICU_HIP_TRY(expr)                                  \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) return HICU_ERR_HIP;              \
  } while (0)

#define HICU_TRY(expr)                                      \
  do {                                                      \
    int32_t _s = (expr);                                    \
    if (_s < 0) return _s;                                  \
  } while (0)

// Host waits that poll an event instead of blocking in the runtime.  A
// solve waits on the device about a hundred times (each Jacobi sweep's
// convergence sums, each outer iteration's step scalars); a blocking wait
// that falls back to an interrupt adds the host's wake-up latency to every
// one of them.  Polling keeps the calling thread busy during the wait.
struct HostWait {
  hipEvent_t e = nullptr;
  HostWait() = default;
  HostWait(const HostWait&) = delete;
  HostWait& operator=(const HostWait&) = delete;
  ~HostWait() {
    if (e) (void)hipEventDestroy(e);
  }
  hipError_t init() { return e ? hipSuccess : hipEventCreateWithFlags(&e, hipEventDisableTiming); }
  // until the last record of e has completed
  hipError_t poll() const {
    hipError_t q;
    while ((q = hipEventQuery(e)) == hipErrorNotReady) {
    }
    return q;
  }
  // until everything queued on st so far has completed
  hipError_t stream(hipStream_t st) {
    hipError_t r = init();
    if (r == hipSuccess) r = hipEventRecord(e, st);
    return r == hipSuccess ? poll() : r;
  }
};

// ---------------------------------------------------------------------------
// Canonical (right-aligned, 3-axis) geometry
// ---------------------------------------------------------------------------
struct Geo {
  int64_t d[3];   // array extents
  int nc;         // coils
  int k[3];       // kernel box
  int64_t lo[3], hi[3];
  int64_t m[3];   // valid extents of region: hi - lo - k + 1
  int wrap[3];    // 1: circular along this axis (whole axis, m = d)
  int kmasked;    // 1: taps restricted to the set bits of kbits (box offsets, lexicographic)
  uint64_t kbits[8];
  int nbox;       // taps of the whole box k0 k1 k2 nc (= n when not masked)
  int64_t s;      // number of valid outputs
  int64_t npts;   // spatial points of the array
  int n;          // taps = k0 k1 k2 nc
};

int32_t make_geo(const hicu_geom* g, Geo* out);
// The same geometry over the whole kernel box (no mask).
Geo box_geo(const Geo& g);
// Device helpers for kernel masks: box offset of the t-th tap, and the tap
// number of box offset f (-1 when f is outside the mask).
__host__ __device__ inline int kmask_tap_of(const uint64_t* bits, int f) {
  if (!((bits[f >> 6] >> (f & 63)) & 1ull)) return -1;
  int t = 0;
  for (int w = 0; w < (f >> 6); ++w) t += __builtin_popcountll(bits[w]);
  const uint64_t low = (f & 63) ? (bits[f >> 6] & ((1ull << (f & 63)) - 1ull)) : 0ull;
  return t + __builtin_popcountll(low);
}
__host__ __device__ inline int kmask_offset_of(const uint64_t* bits, int t) {
  for (int w = 0; w < 8; ++w) {
    const int c = __builtin_popcountll(bits[w]);
    if (t < c) {
      uint64_t v = bits[w];
      for (int i = 0; i < t; ++i) v &= v - 1ull;  // drop the t lowest set bits
      return 64 * w + __builtin_ctzll(v);
    }
    t -= c;
  }
  return -1;
}

// ---------------------------------------------------------------------------
// Precision modes of the contraction kernels
// ---------------------------------------------------------------------------
enum { P_F32 = 0, P_BF16 = 1, P_BF16X3 = 2, P_F16 = 3 };

// Reduction elements per k-block: FP32 uses four 16x16x4 MFMAs per block of
// 16, BF16 one 16x16x32 MFMA per block of 32.
__host__ __device__ constexpr int kblock_of(int prec) { return prec == P_F32 ? 16 : 32; }

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));

// FP32 -> BF16 bits, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ double warp_sum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic block reduction of one double per thread (blockDim.x <= 1024,
// multiple of 64).  Result valid in thread 0.
__device__ __forceinline__ double block_sum_d(double v, double* sh) {
  v = warp_sum_d(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t rup(int64_t a, int64_t b) { return cdiv(a, b) * b; }

}  // namespace hicu
