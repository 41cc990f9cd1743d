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
//
// Shift-correlation route (the default for up to 32 coils).  The entry for
// taps k and k' = k + d only depends on the shift d and on the window
// W_k = {u + k : u valid} of summation points:
//   G[(k,c),(k+d,c')] = sum_{w in W_k} conj(x[w,c]) x[w+d,c'].
// Along each axis the K windows [lo+k, lo+k+m) share their interior, so the
// region splits into segments (single planes near both ends and one core
// segment), every window is a union of K consecutive segments, and the
// region into cells (products of segments).  One pass over the region
// computes, for every cell and every shift d >= 0 (lexicographic order; the
// rest of G follows by Hermitian symmetry), the coil-by-coil correlation sum
// of the cell on the FP64 matrix cores; G is then assembled from the cell
// sums of each window in a fixed order.  Every product is formed exactly as
// in the direct route (FP32 values widened to FP64), only the grouping of
// the sums differs, and the work falls from n^2 s / 2 complex products to
// (2K-1)^D / 2 shifts x Nc^2 coil pairs x |S| points.
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "gram.h"
#include "step.h"

namespace hicu {

// Positions (steps of 4) fetched ahead of the MFMAs that use them.
constexpr int kGramAhead = 8;
constexpr int kCorrAhead = 6;

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



// ---------------------------------------------------------------------------
// Shift-correlation route
// ---------------------------------------------------------------------------

// Route of launch_gram: 1 = shift correlation (when the coil count allows),
// 0 = direct products over the upper block triangle.  Process-wide.
static std::atomic<int> g_route{1};
int gram_route() { return g_route.load(); }
void set_gram_route(int r) { g_route.store(r == 0 ? 0 : 1); }

// Segments of one axis of the region [lo, lo + m + K - 1): with m >= K, K - 1
// single planes, the core [lo + K - 1, lo + m) and K - 1 single planes, and
// window k is segments [k, k + K); with m < K every plane is a segment and
// window k is segments [k, k + m).  A circular axis is one segment (the
// whole axis, m = its extent) shared by every window.
struct AxisSegs {
  int64_t lo, m;
  int K;
  int wrap;
  __host__ __device__ int count() const { return wrap ? 1 : (m >= K ? 2 * K - 1 : (int)(m + K - 1)); }
  __host__ __device__ int64_t start(int j) const {
    if (wrap || m < K) return lo + j;
    return j < K ? lo + j : lo + m + (j - K);
  }
  __host__ __device__ int64_t len(int j) const {
    return wrap ? m : ((m >= K && j == K - 1) ? m - K + 1 : 1);
  }
  // segments of window k: [first(k), first(k) + width())
  __host__ __device__ int first(int k) const { return wrap ? 0 : k; }
  __host__ __device__ int width() const { return wrap ? 1 : (m >= K ? K : (int)m); }
};

struct CorrArgs {
  const float* x;
  int64_t d1, d2;          // array extents of axes 1, 2
  int nc;
  int64_t lo[3], hi[3];    // region
  int64_t per[3];          // period of a circular axis (its extent), 0 otherwise
  int K[3];
  AxisSegs ax[3];
  int ncell;
  int nd_half;             // shifts d >= 0 (lexicographic)
  int64_t chunk;           // points per work entry
  int nent;                // work entries
  int ne, W;               // W = 16 T real components per tile side, ne = W^2
  int* ent_cell;           // [nent] cell of each entry
  int64_t* ent_q;          // [nent][2] point range of each entry inside its cell box
  int* cell_ent;           // [ncell][2] first entry and entry count
  int* multi_cell;         // cells with several entries, in cell order
  double* part;            // [nent][nd_half][ne]  real-embedding partial sums
  double* cellsum;         // [ncell][nd_half][ne] (cells with several entries)
};

__host__ __device__ inline void cell_box(const CorrArgs& a, int cell, int64_t* st, int64_t* ln) {
  const int n2 = a.ax[2].count(), n1 = a.ax[1].count();
  const int j2 = cell % n2, j1 = (cell / n2) % n1, j0 = cell / (n2 * n1);
  st[0] = a.ax[0].start(j0);
  st[1] = a.ax[1].start(j1);
  st[2] = a.ax[2].start(j2);
  ln[0] = a.ax[0].len(j0);
  ln[1] = a.ax[1].len(j1);
  ln[2] = a.ax[2].len(j2);
}

// Work entries: each cell's points (row-major inside the cell box) in chunks
// of a.chunk, numbered cell by cell.  Each of the 256 threads takes a run of
// consecutive cells, counts their entries, and writes them from its
// exclusive prefix (a scan over the threads' counts in LDS); the cells with
// several entries are listed the same way for the reduction.
constexpr int kCorrPlanThreads = 256;
__global__ __launch_bounds__(kCorrPlanThreads) void corr_plan_kernel(CorrArgs a) {
  __shared__ int pre[kCorrPlanThreads], pre_multi[kCorrPlanThreads];
  const int tid = threadIdx.x;
  const int per = (a.ncell + kCorrPlanThreads - 1) / kCorrPlanThreads;
  const int c0 = min(a.ncell, tid * per), c1 = min(a.ncell, c0 + per);
  auto count_of = [&](int c, int64_t* np) {
    int64_t st[3], ln[3];
    cell_box(a, c, st, ln);
    *np = ln[0] * ln[1] * ln[2];
    return (int)((*np + a.chunk - 1) / a.chunk);
  };
  int mine = 0, mine_multi = 0;
  for (int c = c0; c < c1; ++c) {
    int64_t np;
    const int cnt = count_of(c, &np);
    mine += cnt;
    mine_multi += cnt > 1;
  }
  pre[tid] = mine;
  pre_multi[tid] = mine_multi;
  __syncthreads();
  // inclusive scans (Hillis-Steele), then shifted to exclusive
  for (int off = 1; off < kCorrPlanThreads; off <<= 1) {
    const int v = tid >= off ? pre[tid - off] : 0;
    const int vm = tid >= off ? pre_multi[tid - off] : 0;
    __syncthreads();
    pre[tid] += v;
    pre_multi[tid] += vm;
    __syncthreads();
  }
  int e = pre[tid] - mine, mi = pre_multi[tid] - mine_multi;
  for (int c = c0; c < c1; ++c) {
    int64_t np;
    const int cnt = count_of(c, &np);
    a.cell_ent[2 * c] = e;
    a.cell_ent[2 * c + 1] = cnt;
    if (cnt > 1) a.multi_cell[mi++] = c;
    for (int i = 0; i < cnt; ++i, ++e) {
      a.ent_cell[e] = c;
      a.ent_q[2 * e] = (int64_t)i * a.chunk;
      a.ent_q[2 * e + 1] = min(np, (int64_t)(i + 1) * a.chunk);
    }
  }
}

// Shift number h (0 = zero shift) -> d, in lexicographic order of d >= 0.
__host__ __device__ inline void shift_of(const CorrArgs& a, int h, int* d) {
  const int w2 = 2 * a.K[2] - 1, w1 = 2 * a.K[1] - 1, w0 = 2 * a.K[0] - 1;
  const int dl = h + (w0 * w1 * w2 - 1) / 2;
  d[2] = dl % w2 - (a.K[2] - 1);
  d[1] = (dl / w2) % w1 - (a.K[1] - 1);
  d[0] = dl / (w2 * w1) - (a.K[0] - 1);
}

// Shifts per wave: a wave loads its points' components once and pairs them
// with the shifted points of DW shifts, so narrow coil counts (T = 1, 2)
// issue several MFMAs per operand load.
__host__ __device__ constexpr int corr_dw(int T) { return T == 1 ? 4 : (T == 2 ? 2 : 1); }
__host__ __device__ inline int corr_groups(int nd_half, int T) { return (nd_half + 4 * corr_dw(T) - 1) / (4 * corr_dw(T)); }

// Workgroup = (entry, group of 4 DW shifts); wave v takes the DW shifts from
// (4 group + v) DW and accumulates, for each, the T x T grid of 16 x 16
// real-embedding tiles of sum_w x[w] x[w + d]^T with v_mfma_f64_16x16x4
// (4 points per step; lane group g takes points g, g + 4, ...).  x[w + d]
// outside the region counts as zero (such cell/shift pairs are never
// assembled); on a circular axis it wraps.  Operands are fetched kCorrAhead
// steps ahead and widened to FP64 at use.
template <int T>
__global__ __launch_bounds__(256) void corr_kernel(CorrArgs a) {
  constexpr int DW = corr_dw(T);
  const int ngrp = corr_groups(a.nd_half, T);
  // Workgroups are dealt to the 8 XCDs in turn.  Entry e runs on XCD
  // e mod 8 with all its shift groups there back to back: neighbouring
  // entries have similar sizes, so every XCD gets an even share of the
  // heavy core entries, and the groups of one entry share an L2.  (Giving
  // each XCD a contiguous range of entries instead put the whole core cell
  // on one or two XCDs.)
  const int64_t xcd = blockIdx.x % 8, idx = blockIdx.x / 8;
  const int ent = (int)((idx / ngrp) * 8 + xcd), grp = (int)(idx % ngrp);
  if (ent >= a.nent) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, m = lane & 15;
  const int h0 = (grp * 4 + wave) * DW;
  if (h0 >= a.nd_half) return;
  int d[DW][3];
  bool hok[DW];
#pragma unroll
  for (int u = 0; u < DW; ++u) {
    hok[u] = h0 + u < a.nd_half;
    shift_of(a, hok[u] ? h0 + u : h0, d[u]);
  }
  int64_t cst[3], cln[3];
  cell_box(a, a.ent_cell[ent], cst, cln);
  const int64_t q_begin = a.ent_q[2 * ent], q_end = a.ent_q[2 * ent + 1];
  const int two_nc = 2 * a.nc;
  bool okc[T];
#pragma unroll
  for (int i = 0; i < T; ++i) okc[i] = 16 * i + m < two_nc;

  double4_t acc[DW][T][T];
#pragma unroll
  for (int u = 0; u < DW; ++u)
#pragma unroll
    for (int i = 0; i < T; ++i)
#pragma unroll
      for (int j = 0; j < T; ++j) acc[u][i][j] = double4_t{0.0, 0.0, 0.0, 0.0};

  // Fast path (uniform per wave).  Off circular axes a cell is one plane or
  // the core segment, so a shift moves the whole cell box either inside the
  // region (the core stays inside for every shift) or, on some axis,
  // entirely outside it.  When each of the wave's shifts is one or the
  // other, no index wraps and no bound is checked per point: a shift inside
  // reads at a fixed offset from the unshifted operand, one outside
  // contributes zeros.
  bool fast = true, inb[DW];
  int64_t doff[DW];
#pragma unroll
  for (int u = 0; u < DW; ++u) {
    doff[u] = ((int64_t)d[u][0] * a.d1 * a.d2 + (int64_t)d[u][1] * a.d2 + d[u][2]) * two_nc;
    bool in = true, out = false;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int64_t b0 = cst[ax] + d[u][ax], b1 = cst[ax] + cln[ax] - 1 + d[u][ax];
      in = in && b0 >= a.lo[ax] && b1 < a.hi[ax];
      out = out || (a.per[ax] == 0 && (b1 < a.lo[ax] || b0 >= a.hi[ax]));
    }
    inb[u] = in && hok[u];
    fast = fast && (in || out);
  }
  int64_t q = q_begin + g;
  int64_t p2 = q % cln[2], p1 = (q / cln[2]) % cln[1], p0 = q / (cln[2] * cln[1]);
  auto base_of = [&]() { return (((cst[0] + p0) * a.d1 + (cst[1] + p1)) * a.d2 + (cst[2] + p2)) * two_nc; };
  int64_t base = base_of();
  // A lane past the entry's end reads at the entry's first point instead
  // (in the region, and so is each of its in-region shifts); masked-off
  // components read component 0.  Loads carry no select: the masks are
  // applied where the values are used, so the compiler never has to wait
  // for a load before the ring moves on.
  const int64_t base_first = (((cst[0] + q_begin / (cln[2] * cln[1])) * a.d1 + (cst[1] + (q_begin / cln[2]) % cln[1])) *
                                  a.d2 + (cst[2] + q_begin % cln[2])) * two_nc;
  int offc[T];
#pragma unroll
  for (int i = 0; i < T; ++i) offc[i] = okc[i] ? 16 * i + m : 0;
  // Shifts out of the region read the unshifted point (their values are
  // masked to zero).  The empty asm hides that from the optimiser, which
  // would otherwise reuse the unshifted load for such shifts and so wait
  // for that load in the step that issues it.
  int64_t soff[DW];
#pragma unroll
  for (int u = 0; u < DW; ++u) {
    soff[u] = inb[u] ? doff[u] : 0;
    asm volatile("" : "+v"(soff[u]));
  }
  auto wrap_to = [](int64_t v, int64_t P) { return P == 0 ? v : (v < 0 ? v + P : (v >= P ? v - P : v)); };
  // The two paths get separate loops, so the fast one carries no wrap or
  // bound logic.  The slow path keeps a per-slot bit mask (bit u: shift u's
  // point lies in the region).
  auto run = [&](auto fast_tag) {
    constexpr bool FAST = decltype(fast_tag)::value;
    auto fetch = [&](float (&av)[T], float (&bv)[DW][T], unsigned& mk) {
      const bool ok = q < q_end;
      if constexpr (FAST) {
        const int64_t b = ok ? base : base_first;
#pragma unroll
        for (int i = 0; i < T; ++i) av[i] = a.x[b + offc[i]];
#pragma unroll
        for (int u = 0; u < DW; ++u)
#pragma unroll
          for (int i = 0; i < T; ++i) bv[u][i] = a.x[b + soff[u] + offc[i]];
        mk = 0;
      } else {
#pragma unroll
        for (int i = 0; i < T; ++i) av[i] = a.x[(ok ? base : base_first) + offc[i]];
        const int64_t w0 = cst[0] + p0, w1 = cst[1] + p1, w2 = cst[2] + p2;
        mk = 0;
#pragma unroll
        for (int u = 0; u < DW; ++u) {
          const int64_t v0 = wrap_to(w0 + d[u][0], a.per[0]), v1 = wrap_to(w1 + d[u][1], a.per[1]),
                        v2 = wrap_to(w2 + d[u][2], a.per[2]);
          const bool okb = ok && hok[u] && v0 >= a.lo[0] && v0 < a.hi[0] && v1 >= a.lo[1] && v1 < a.hi[1] &&
                           v2 >= a.lo[2] && v2 < a.hi[2];
          const int64_t bbase = okb ? ((v0 * a.d1 + v1) * a.d2 + v2) * two_nc : base_first;
          mk |= okb ? 1u << u : 0u;
#pragma unroll
          for (int i = 0; i < T; ++i) bv[u][i] = a.x[bbase + offc[i]];
        }
      }
      q += 4;
      p2 += 4;
      if (p2 < cln[2]) {
        base += 4 * two_nc;
      } else {
        while (p2 >= cln[2]) {
          p2 -= cln[2];
          if (++p1 == cln[1]) {
            p1 = 0;
            ++p0;
          }
        }
        base = base_of();
      }
    };
    constexpr int PF = kCorrAhead;
    float av[PF][T], bv[PF][DW][T];
    unsigned mk[PF];
#pragma unroll
    for (int r = 0; r < PF; ++r) fetch(av[r], bv[r], mk[r]);
    // Whole blocks of PF steps: steps past the entry's end see all-zero
    // operands (their lanes are masked), which keeps the block free of
    // exits.
    for (int64_t q0 = q_begin; q0 < q_end; q0 += 4 * PF) {
#pragma unroll
      for (int r = 0; r < PF; ++r) {
        // masks as factors 1 or 0: a select on a loaded value would make
        // the compiler wait for (or predicate) the load where it is issued
        const bool ok = q0 + 4 * r + g < q_end;
        double ad[T];
#pragma unroll
        for (int i = 0; i < T; ++i) ad[i] = (double)(av[r][i] * (ok && okc[i] ? 1.f : 0.f));
#pragma unroll
        for (int u = 0; u < DW; ++u) {
          const bool okb = FAST ? ok && inb[u] : ((mk[r] >> u) & 1u) != 0;
          double bd[T];
#pragma unroll
          for (int j = 0; j < T; ++j) bd[j] = (double)(bv[r][u][j] * (okb && okc[j] ? 1.f : 0.f));
#pragma unroll
          for (int i = 0; i < T; ++i)
#pragma unroll
            for (int j = 0; j < T; ++j)
              acc[u][i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ad[i], bd[j], acc[u][i][j], 0, 0, 0);
        }
        fetch(av[r], bv[r], mk[r]);  // the step PF positions further on
      }
    }
  };
  if (fast) run(std::true_type{});
  else run(std::false_type{});
  // v_mfma_f64_16x16x4: lane holds rows g, g + 4, g + 8, g + 12 of column m
#pragma unroll
  for (int u = 0; u < DW; ++u) {
    if (!hok[u]) continue;
    double* out = a.part + ((size_t)ent * a.nd_half + h0 + u) * a.ne;
#pragma unroll
    for (int i = 0; i < T; ++i)
#pragma unroll
      for (int j = 0; j < T; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(16 * i + g + 4 * r) * a.W + 16 * j + m] = acc[u][i][j][r];
  }
}

// Cells split over several entries (grid axis y walks their list): their
// partial sums added in entry order.
__global__ __launch_bounds__(256) void corr_reduce_kernel(CorrArgs a) {
  const int cell = a.multi_cell[blockIdx.y];
  const int first = a.cell_ent[2 * cell], cnt = a.cell_ent[2 * cell + 1];
  const int64_t per = (int64_t)a.nd_half * a.ne;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < per; e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < cnt; ++i) s += a.part[(size_t)(first + i) * per + e];
    a.cellsum[(size_t)cell * per + e] = s;
  }
}

// G from the cell sums: one thread per (tap k, shift h, coil pair); the
// window W_k is the product of each axis's segments [k_a, k_a + width),
// summed in cell order; the mirrored entry is the conjugate, so G is exactly
// Hermitian with a real diagonal.
__global__ __launch_bounds__(256) void corr_assemble_kernel(CorrArgs a, int n, double2* G) {
  const int nc = a.nc;
  const int64_t total = (int64_t)a.K[0] * a.K[1] * a.K[2] * a.nd_half * nc * nc;
  const int64_t per = (int64_t)a.nd_half * a.ne;
  const int n2 = a.ax[2].count(), n1 = a.ax[1].count();
  const int wd0 = a.ax[0].width(), wd1 = a.ax[1].width(), wd2 = a.ax[2].width();
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int cp = (int)(t % nc), c = (int)((t / nc) % nc);
    const int h = (int)((t / ((int64_t)nc * nc)) % a.nd_half);
    const int kl = (int)(t / ((int64_t)nc * nc * a.nd_half));
    const int k2 = kl % a.K[2], k1 = (kl / a.K[2]) % a.K[1], k0 = kl / (a.K[2] * a.K[1]);
    int d[3];
    shift_of(a, h, d);
    const int q0 = k0 + d[0], q1 = k1 + d[1], q2 = k2 + d[2];
    if (q0 < 0 || q0 >= a.K[0] || q1 < 0 || q1 >= a.K[1] || q2 < 0 || q2 >= a.K[2]) continue;
    if (h == 0 && cp < c) continue;  // zero shift: upper triangle of the coil block, mirrored below
    double rr = 0.0, ii = 0.0, ri = 0.0, ir = 0.0;
    const int e_rr = (2 * c) * a.W + 2 * cp, e_ii = (2 * c + 1) * a.W + 2 * cp + 1;
    const int e_ri = (2 * c) * a.W + 2 * cp + 1, e_ir = (2 * c + 1) * a.W + 2 * cp;
    const int f0 = a.ax[0].first(k0), f1 = a.ax[1].first(k1), f2 = a.ax[2].first(k2);
    for (int j0 = f0; j0 < f0 + wd0; ++j0)
      for (int j1 = f1; j1 < f1 + wd1; ++j1)
        for (int j2 = f2; j2 < f2 + wd2; ++j2) {
          const int cell = (j0 * n1 + j1) * n2 + j2;
          const int first = a.cell_ent[2 * cell], cnt = a.cell_ent[2 * cell + 1];
          const double* src =
              (cnt > 1 ? a.cellsum + (size_t)cell * per : a.part + (size_t)first * per) + (size_t)h * a.ne;
          rr += src[e_rr];
          ii += src[e_ii];
          ri += src[e_ri];
          ir += src[e_ir];
        }
    const int i = kl * nc + c, jj = ((q0 * a.K[1] + q1) * a.K[2] + q2) * nc + cp;
    const double re = rr + ii, im = i == jj ? 0.0 : ri - ir;
    G[(size_t)i * n + jj] = make_double2(re, im);
    if (i != jj) G[(size_t)jj * n + i] = make_double2(re, -im);
  }
}

namespace {

constexpr int kCorrMaxCoils = 32;  // T <= 4 tiles of 16 real components

struct CorrPlan {
  CorrArgs a;
  int T;
  size_t off_ent_cell, off_ent_q, off_cell_ent, off_multi, off_part, off_cellsum, total;
  int multi;  // cells with several entries
};

bool corr_plan(const Geo& g, CorrPlan* p) {
  if (g.nc > kCorrMaxCoils) return false;
  CorrArgs& a = p->a;
  a = CorrArgs{};
  a.nc = g.nc;
  a.d1 = g.d[1];
  a.d2 = g.d[2];
  for (int i = 0; i < 3; ++i) {
    a.lo[i] = g.lo[i];
    a.hi[i] = g.hi[i];
    a.K[i] = g.k[i];
    a.ax[i].lo = g.lo[i];
    a.ax[i].m = g.m[i];
    a.ax[i].K = g.k[i];
    a.ax[i].wrap = g.wrap[i];
    a.per[i] = g.wrap[i] ? g.d[i] : 0;
  }
  a.ncell = a.ax[0].count() * a.ax[1].count() * a.ax[2].count();
  if (a.ncell > 65535) return false;  // the reduce launch puts cells on grid axis y
  a.nd_half = ((2 * g.k[0] - 1) * (2 * g.k[1] - 1) * (2 * g.k[2] - 1) + 1) / 2;
  p->T = (int)cdiv(2 * g.nc, 16);
  a.W = 16 * p->T;
  a.ne = a.W * a.W;
  const int64_t npts = region_points(g);
  // entries sized for about 2048 heavy workgroups (several waves per SIMD to
  // hide the operand loads), at least 512 points each
  a.chunk = std::max<int64_t>(512, std::min<int64_t>(131072, rup(npts * corr_groups(a.nd_half, p->T) / 2048, 4)));
  int64_t nent = 0, multi = 0;
  for (int c = 0; c < a.ncell; ++c) {
    int64_t st[3], ln[3];
    cell_box(a, c, st, ln);
    const int64_t k = cdiv(ln[0] * ln[1] * ln[2], a.chunk);
    nent += k;
    multi += k > 1;
  }
  const int64_t ngrp = corr_groups(a.nd_half, p->T);
  if (nent > (1 << 24) || nent * ngrp > 0x7fffffffLL) return false;
  a.nent = (int)nent;
  const size_t per = (size_t)a.nd_half * a.ne * sizeof(double);
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += (b + 255) / 256 * 256;
    return o;
  };
  p->off_ent_cell = take((size_t)nent * sizeof(int));
  p->off_ent_q = take(2 * (size_t)nent * sizeof(int64_t));
  p->off_cell_ent = take(2 * (size_t)a.ncell * sizeof(int));
  p->off_multi = take((size_t)a.ncell * sizeof(int));
  p->multi = (int)multi;
  p->off_part = take((size_t)nent * per);
  p->off_cellsum = take(multi > 0 ? (size_t)a.ncell * per : 0);
  p->total = off;
  return true;
}

}  // namespace

// Kernel mask: G[i][j] = Gbox[box(i)][box(j)], box(t c) = (box offset of
// tap t) nc + c.
struct KBits {
  uint64_t w[8];
};
__global__ __launch_bounds__(256) void gram_select_kernel(const double2* Gbox, int nbox, KBits bits, int nc, int n,
                                                          double2* G) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    const int bi = kmask_offset_of(bits.w, i / nc) * nc + i % nc;
    const int bj = kmask_offset_of(bits.w, j / nc) * nc + j % nc;
    G[e] = Gbox[(size_t)bi * nbox + bj];
  }
}

static int32_t launch_gram_box(const Geo& g, const void* x, void* G, void* ws, size_t ws_bytes, hipStream_t st);

int32_t launch_gram(const Geo& g, const void* x, void* G, void* ws, size_t ws_bytes, hipStream_t st) {
  if (!g.kmasked) return launch_gram_box(g, x, G, ws, ws_bytes, st);
  const Geo b = box_geo(g);
  const size_t gb = al((size_t)g.nbox * g.nbox * sizeof(double2));
  if (ws == nullptr || ws_bytes < gb) return HICU_ERR_WORKSPACE;
  HICU_TRY(launch_gram_box(b, x, ws, at(ws, gb), ws_bytes - gb, st));
  KBits kb;
  for (int w = 0; w < 8; ++w) kb.w[w] = g.kbits[w];
  const int64_t tot = (int64_t)g.n * g.n;
  hipLaunchKernelGGL(gram_select_kernel, dim3((unsigned)std::min<int64_t>(cdiv(tot, 256), 16384)), dim3(256), 0, st,
                     reinterpret_cast<const double2*>(ws), g.nbox, kb, g.nc, g.n, reinterpret_cast<double2*>(G));
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

static int32_t launch_gram_box(const Geo& g, const void* x, void* G, void* ws, size_t ws_bytes, hipStream_t st) {
  CorrPlan cp;
  const bool circular = g.wrap[0] || g.wrap[1] || g.wrap[2];
  if ((gram_route() == 1 || circular) && corr_plan(g, &cp)) {
    if (ws == nullptr || ws_bytes < cp.total) return HICU_ERR_WORKSPACE;
    CorrArgs a = cp.a;
    char* b = reinterpret_cast<char*>(ws);
    a.x = reinterpret_cast<const float*>(x);
    a.ent_cell = reinterpret_cast<int*>(b + cp.off_ent_cell);
    a.ent_q = reinterpret_cast<int64_t*>(b + cp.off_ent_q);
    a.cell_ent = reinterpret_cast<int*>(b + cp.off_cell_ent);
    a.multi_cell = reinterpret_cast<int*>(b + cp.off_multi);
    a.part = reinterpret_cast<double*>(b + cp.off_part);
    a.cellsum = reinterpret_cast<double*>(b + cp.off_cellsum);
    hipLaunchKernelGGL(corr_plan_kernel, dim3(1), dim3(kCorrPlanThreads), 0, st, a);
    const int ngrp = corr_groups(a.nd_half, cp.T);
    const dim3 grid((unsigned)(rup((int64_t)a.nent, 8) * ngrp));
    switch (cp.T) {
      case 1: hipLaunchKernelGGL(corr_kernel<1>, grid, dim3(256), 0, st, a); break;
      case 2: hipLaunchKernelGGL(corr_kernel<2>, grid, dim3(256), 0, st, a); break;
      case 3: hipLaunchKernelGGL(corr_kernel<3>, grid, dim3(256), 0, st, a); break;
      default: hipLaunchKernelGGL(corr_kernel<4>, grid, dim3(256), 0, st, a); break;
    }
    const int64_t per = (int64_t)a.nd_half * a.ne;
    if (cp.multi > 0)
      hipLaunchKernelGGL(corr_reduce_kernel, dim3((unsigned)std::min<int64_t>(cdiv(per, 256), 1024), cp.multi),
                         dim3(256), 0, st, a);
    const int64_t tot = (int64_t)g.k[0] * g.k[1] * g.k[2] * a.nd_half * g.nc * g.nc;
    hipLaunchKernelGGL(corr_assemble_kernel, dim3((unsigned)std::min<int64_t>(cdiv(tot, 256), 65536)), dim3(256), 0,
                       st, a, g.n, reinterpret_cast<double2*>(G));
    HICU_HIP_TRY(hipGetLastError());
    return HICU_OK;
  }
  if (circular) return HICU_ERR_UNSUPPORTED;  // the direct route has no circular axes
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

size_t gram_workspace(const Geo& g) {
  if (g.kmasked) return al((size_t)g.nbox * g.nbox * sizeof(double2)) + gram_workspace(box_geo(g));
  int ntile, ntri, ngroups;
  int64_t qper;
  gram_layout(g, &ntile, &ntri, &ngroups, &qper);
  const size_t direct = (size_t)ngroups * ntri * 4096 * sizeof(double);
  CorrPlan cp;
  return std::max(direct, corr_plan(g, &cp) ? cp.total : (size_t)0);
}

}  // namespace hicu
