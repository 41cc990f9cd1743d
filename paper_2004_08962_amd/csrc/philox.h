// Device-side counter-based normals and the JL product shared by the
// single-problem and the batched kernels (one definition, so both draw and
// sum identically).
#pragma once

#include "common.h"

namespace hicu {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; each round
// multiplies counter words 0 and 2 by the two Philox multipliers, mixes the
// high halves with words 1, 3 and the round key, and bumps the key by the
// two Weyl increments.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Standard normal number `e` of the stream (seed, outer, inner, stream_id):
// block e/4 of Philox, words mapped to u = (w + 1/2) 2^-32, Box-Muller on
// (w0, w1) -> z0, z1 and (w2, w3) -> z2, z3.
__device__ __forceinline__ double philox_normal(int64_t e, uint64_t seed, uint32_t outer, uint32_t inner,
                                                uint32_t sid) {
  uint32_t c[4] = {(uint32_t)(e >> 2), outer, inner, sid};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const int lane = (int)(e & 3);
  const double two32 = 2.3283064365386963e-10;  // 2^-32
  const double ua = ((double)c[lane < 2 ? 0 : 2] + 0.5) * two32;
  const double ub = ((double)c[lane < 2 ? 1 : 3] + 0.5) * two32;
  const double R = sqrt(-2.0 * log(ua));
  const double ang = 2.0 * 3.14159265358979323846 * ub;
  return (lane & 1) ? R * sin(ang) : R * cos(ang);
}

// Rows per workgroup of the JL product (four waves of 16 rows).
constexpr int kJlRows = 64;

// Column j of F = Q P for rows [row0, row0 + kJlRows): P[:, j] (nq values,
// N(0, 1/p)) is drawn into pcol by the whole block, then each wave forms 16
// rows, its lanes striding over l (coalesced reads of a row of Q, FP64
// sums) and a fixed-order wave reduction giving each entry.  Pout (optional)
// receives P[:, j] from the block of row 0.
__device__ __forceinline__ void jl_column_rows(const float2* Q, int n, int nq, int p, int j, int row0,
                                               uint64_t seed, uint32_t outer, uint32_t inner, uint32_t sid,
                                               double* pcol, float2* F, double* Pout) {
  const double scale = 1.0 / sqrt((double)p);
  for (int l = threadIdx.x; l < nq; l += blockDim.x) {
    const double v = philox_normal((int64_t)l * p + j, seed, outer, inner, sid) * scale;
    pcol[l] = v;
    if (Pout && row0 == 0) Pout[(size_t)l * p + j] = v;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int rr = 0; rr < kJlRows / 4; ++rr) {
    const int i = row0 + wave * (kJlRows / 4) + rr;
    if (i >= n) break;
    const float2* q = Q + (size_t)i * nq;
    double re = 0.0, im = 0.0;
    for (int l = lane; l < nq; l += 64) {
      const float2 v = q[l];
      re += (double)v.x * pcol[l];
      im += (double)v.y * pcol[l];
    }
    re = warp_sum_d(re);
    im = warp_sum_d(im);
    if (lane == 0) F[(size_t)i * p + j] = make_float2((float)re, (float)im);
  }
}

}  // namespace hicu
