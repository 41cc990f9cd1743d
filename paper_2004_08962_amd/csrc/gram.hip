// Gram matrix G = H_S(x)' H_S(x) on the FP64 matrix cores.
//
// DISCUSSION section: the nullspace can be taken from the Gram matrix of the
// multi-level Hankel matrix instead of an rSVD.  With the real embedding of
// the interleaved complex data, Gr = A^T A where row u of A holds the
// (re, im) entries of the patch at valid output u; the complex Gram follows
// as Re G = Gr[re,re] + Gr[im,im], Im G = Gr[re,im] - Gr[im,re].
// Each block owns one 64 x 64 tile of the upper block triangle of Gr and a
// contiguous range of positions; operands are fetched from L1/L2 (16 lanes
// read 16 consecutive floats), widened to FP64 and accumulated by
// v_mfma_f64_16x16x4.  Per-range partial tiles are summed in a fixed order
// by a second kernel, so the result is deterministic.
#include <algorithm>

#include "gram.h"

namespace hicu {

// Positions (steps of 4) fetched ahead of the MFMAs that use them.
constexpr int kGramAhead = 8;

struct GramArgs {
  const float* x;       // complex64 array viewed as floats
  int64_t d1, d2;       // array extents of axes 1, 2
  int nc;
  int k0, k1, k2;
  int64_t lo[3];
  int64_t m1, m2;       // valid extents of axes 1, 2
  int64_t s;            // valid outputs
  int nr;               // real Gram dimension 2n
  int ntile;            // 64-wide tiles per dimension
  int ntri;             // upper-triangle tile count
  int64_t qper;         // positions per block (multiple of 4)
  int ngroups;          // position ranges
  double* part;         // [ngroups][ntri][64][64]
};

__device__ __forceinline__ void tri_index(int t, int ntile, int* I, int* J) {
  int i = 0;
  while (t >= ntile - i) {
    t -= ntile - i;
    ++i;
  }
  *I = i;
  *J = i + t;
}

__device__ __forceinline__ int64_t real_row_offset(const GramArgs& a, int e) {
  // e = kk * (2 nc) + el  ->  float offset 2 nc * pt(kk) + el
  const int two_nc = 2 * a.nc;
  const int kk = e / two_nc, el = e % two_nc;
  const int kk2 = kk % a.k2, kk1 = (kk / a.k2) % a.k1, kk0 = kk / (a.k2 * a.k1);
  const int64_t pt = ((int64_t)kk0 * a.d1 + kk1) * a.d2 + kk2;
  return pt * two_nc + el;
}

// Work item w of W = ntri * ngroups -> linear item: workgroups reach the 8
// XCDs round-robin, so the id is remapped to give each XCD a contiguous run
// of items.  Items are ordered range-major, so the tiles that read the same
// positions run together and share that XCD's L2.
__device__ __forceinline__ int64_t gram_remap(int64_t w, int64_t W) {
  const int64_t per = W / 8, rem = W % 8;
  const int64_t xcd = w % 8, idx = w / 8;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

__global__ __launch_bounds__(256) void gram_tile_kernel(GramArgs a) {
  const int64_t lin = gram_remap(blockIdx.x, (int64_t)a.ntri * a.ngroups);
  const int tile = (int)(lin % a.ntri), grp = (int)(lin / a.ntri);
  int I, J;
  tri_index(tile, a.ntile, &I, &J);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, m = lane & 15;
  const int wr = wave >> 1, wc = wave & 1;

  int64_t offA[2], offB[2];
  bool okA[2], okB[2];
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    const int ea = I * 64 + wr * 32 + f * 16 + m;
    const int eb = J * 64 + wc * 32 + f * 16 + m;
    okA[f] = ea < a.nr;
    okB[f] = eb < a.nr;
    offA[f] = okA[f] ? real_row_offset(a, ea) : 0;
    offB[f] = okB[f] ? real_row_offset(a, eb) : 0;
  }

  double4_t acc[2][2];
#pragma unroll
  for (int f = 0; f < 2; ++f)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[f][j] = double4_t{0.0, 0.0, 0.0, 0.0};

  const int64_t q_begin = (int64_t)grp * a.qper;
  const int64_t q_end = std::min<int64_t>(a.s, q_begin + a.qper);
  const int64_t two_nc = 2 * a.nc;
  // Lane group g walks positions q_begin + g, + 4, ...: its output index
  // (u0, u1, u2) and float offset advance incrementally (a carry into u1 /
  // u0 recomputes the offset).  Operands are fetched kGramAhead positions
  // ahead into a register ring and widened to FP64 only when used, so the
  // loads stay in flight across that many steps of MFMAs.
  int64_t q = q_begin + g;
  int64_t u2 = q % a.m2, u1 = (q / a.m2) % a.m1, u0 = q / (a.m2 * a.m1);
  auto offset_of = [&]() {
    return (((a.lo[0] + u0) * a.d1 + (a.lo[1] + u1)) * a.d2 + (a.lo[2] + u2)) * two_nc;
  };
  int64_t base = offset_of();
  auto fetch = [&](float (&av)[2], float (&bv)[2]) {
    const bool ok = q < q_end;
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      av[f] = (ok && okA[f]) ? a.x[base + offA[f]] : 0.f;
      bv[f] = (ok && okB[f]) ? a.x[base + offB[f]] : 0.f;
    }
    q += 4;
    u2 += 4;
    if (u2 < a.m2) {
      base += 4 * two_nc;
    } else {
      while (u2 >= a.m2) {
        u2 -= a.m2;
        if (++u1 == a.m1) {
          u1 = 0;
          ++u0;
        }
      }
      base = offset_of();
    }
  };
  constexpr int PF = kGramAhead;
  float av[PF][2], bv[PF][2];
#pragma unroll
  for (int r = 0; r < PF; ++r) fetch(av[r], bv[r]);
  for (int64_t q0 = q_begin; q0 < q_end; q0 += 4 * PF) {
#pragma unroll
    for (int r = 0; r < PF; ++r) {
      if (q0 + 4 * r >= q_end) break;
      double ad[2], bd[2];
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        ad[f] = (double)av[r][f];
        bd[f] = (double)bv[r][f];
      }
#pragma unroll
      for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[f][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ad[f], bd[j], acc[f][j], 0, 0, 0);
      fetch(av[r], bv[r]);  // the step PF positions further on
    }
  }

  double* out = a.part + ((size_t)grp * a.ntri + tile) * 4096;
#pragma unroll
  for (int f = 0; f < 2; ++f)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // v_mfma_f64_16x16x4: lane holds rows g, g + 4, g + 8, g + 12 of column m
        const int r = wr * 32 + f * 16 + g + 4 * i;
        const int c = wc * 32 + j * 16 + m;
        out[r * 64 + c] = acc[f][j][i];
      }
}

// Sum the partial tiles in order of the position range and scatter the
// complex Gram: the upper triangle is computed and mirrored, so G is exactly
// Hermitian with a real diagonal.
__global__ __launch_bounds__(256) void gram_finalize_kernel(const double* part, int ngroups, int ntri,
                                                            int ntile, int n, double2* G) {
  int I, J;
  tri_index(blockIdx.x, ntile, &I, &J);
  for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
    const int lr = e / 32, lc = e % 32;         // complex offsets inside the tile
    const int i = I * 32 + lr, j = J * 32 + lc;  // complex indices
    if (i >= n || j >= n || (I == J && lc < lr)) continue;
    double rr = 0.0, ii = 0.0, ri = 0.0, ir = 0.0;
    for (int y = 0; y < ngroups; ++y) {
      const double* t = part + ((size_t)y * ntri + blockIdx.x) * 4096;
      rr += t[(2 * lr) * 64 + 2 * lc];
      ii += t[(2 * lr + 1) * 64 + 2 * lc + 1];
      ri += t[(2 * lr) * 64 + 2 * lc + 1];
      ir += t[(2 * lr + 1) * 64 + 2 * lc];
    }
    const double re = rr + ii, im = i == j ? 0.0 : ri - ir;
    G[(size_t)i * n + j] = make_double2(re, im);
    if (i != j) G[(size_t)j * n + i] = make_double2(re, -im);
  }
}

static void gram_layout(const Geo& g, int* ntile, int* ntri, int* ngroups, int64_t* qper) {
  const int nr = 2 * g.n;
  *ntile = (int)cdiv(nr, 64);
  *ntri = *ntile * (*ntile + 1) / 2;
  // Enough blocks to fill 256 CUs several times, at least 64 k-groups each.
  int64_t groups = std::max<int64_t>(1, 4096 / *ntri);
  groups = std::min<int64_t>(groups, std::max<int64_t>(1, g.s / 256));
  *qper = rup(cdiv(g.s, groups), 4);
  *ngroups = (int)cdiv(g.s, *qper);
}

size_t gram_workspace(const Geo& g) {
  int ntile, ntri, ngroups;
  int64_t qper;
  gram_layout(g, &ntile, &ntri, &ngroups, &qper);
  return (size_t)ngroups * ntri * 4096 * sizeof(double);
}

int32_t launch_gram(const Geo& g, const void* x, void* G, void* ws, size_t ws_bytes, hipStream_t st) {
  int ntile, ntri, ngroups;
  int64_t qper;
  gram_layout(g, &ntile, &ntri, &ngroups, &qper);
  const size_t need = (size_t)ngroups * ntri * 4096 * sizeof(double);
  if (ws == nullptr || ws_bytes < need) return HICU_ERR_WORKSPACE;
  GramArgs a;
  a.x = reinterpret_cast<const float*>(x);
  a.d1 = g.d[1];
  a.d2 = g.d[2];
  a.nc = g.nc;
  a.k0 = g.k[0];
  a.k1 = g.k[1];
  a.k2 = g.k[2];
  for (int i = 0; i < 3; ++i) a.lo[i] = g.lo[i];
  a.m1 = g.m[1];
  a.m2 = g.m[2];
  a.s = g.s;
  a.nr = 2 * g.n;
  a.ntile = ntile;
  a.ntri = ntri;
  a.qper = qper;
  a.ngroups = ngroups;
  a.part = reinterpret_cast<double*>(ws);
  if ((int64_t)ntri * ngroups > 0x7fffffff) return HICU_ERR_SHAPE;
  hipLaunchKernelGGL(gram_tile_kernel, dim3((unsigned)(ntri * ngroups)), dim3(256), 0, st, a);
  HICU_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(gram_finalize_kernel, dim3(ntri), dim3(256), 0, st, (const double*)a.part, ngroups,
                     ntri, ntile, g.n, reinterpret_cast<double2*>(G));
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

}  // namespace hicu
