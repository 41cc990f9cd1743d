// Valid multi-channel correlation on the CDNA4 matrix cores.
//
// Every contraction of the gradient step is the same operation: a
// correlation of a channel-fastest input array with a small kernel box that
// sums over all input channels (THEORY section: the Hankel product H(x)v is
// a valid convolution; the kernel spans all coils; the adjoint H' is itself
// a valid convolution).  The block stages a halo tile of the input in LDS
// (one channel chunk at a time) and forms im2col fragments straight from it:
// for fixed kernel offsets (k0, k1) the run over (k2, channel, re/im) is
// contiguous in the tile, so each lane fetches its MFMA operand with one
// 16-byte LDS read.  Weights are pre-arranged in fragment order and read
// from L1/L2 with coalesced 16-byte loads.  Complex arithmetic uses the real
// 2x2 embedding, so the contraction is a plain real GEMM on interleaved
// (re, im) data.
#include <algorithm>

#include "conv.h"

namespace hicu {

template <int PREC> struct LdsElem { using T = float; };
template <> struct LdsElem<P_BF16> { using T = uint16_t; };
template <> struct LdsElem<P_BF16X3> { using T = uint16_t; };

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

typedef float float2v_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));

// Two floats -> packed BF16 (round to nearest even; one v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t pack_bf16(float x, float y) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(float2v_t{x, y}, bf16x2_t));
}
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// Store 2V floats (V complex values, interleaved re/im) at LDS element
// offset off: FP32 as is, BF16 rounded, split BF16 as hi and lo = v - hi.
template <int PREC, int V>
__device__ __forceinline__ void stage_store(typename LdsElem<PREC>::T* hi, typename LdsElem<PREC>::T* lo, int off,
                                            const float (&v)[2 * V]) {
  if constexpr (PREC == P_F32) {
    if constexpr (V == 4) {
      *reinterpret_cast<float4_t*>(hi + off) = float4_t{v[0], v[1], v[2], v[3]};
      *reinterpret_cast<float4_t*>(hi + off + 4) = float4_t{v[4], v[5], v[6], v[7]};
    } else if constexpr (V == 2) {
      *reinterpret_cast<float4_t*>(hi + off) = float4_t{v[0], v[1], v[2], v[3]};
    } else {
      *reinterpret_cast<float2*>(hi + off) = make_float2(v[0], v[1]);
    }
  } else {
    uint32_t w[V], wl[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      w[i] = pack_bf16(v[2 * i], v[2 * i + 1]);
      if constexpr (PREC == P_BF16X3) wl[i] = pack_bf16(v[2 * i] - bf16_lo(w[i]), v[2 * i + 1] - bf16_hi(w[i]));
    }
    auto put = [&](uint16_t* dst, const uint32_t (&x)[V]) {
      if constexpr (V == 4) *reinterpret_cast<u32x4_t*>(dst + off) = u32x4_t{x[0], x[1], x[2], x[3]};
      else if constexpr (V == 2) *reinterpret_cast<u32x2_t*>(dst + off) = u32x2_t{x[0], x[1]};
      else *reinterpret_cast<uint32_t*>(dst + off) = x[0];
    };
    put(hi, w);
    if constexpr (PREC == P_BF16X3) put(lo, wl);
  }
}

// V complex values from global memory at in + idx: nv = V loads them with
// 16-byte loads, 0 < nv < V one by one (the rest zero), nv = 0 gives zeros.
template <int V>
__device__ __forceinline__ void load_unit(const float2* in, int64_t idx, int nv, float (&v)[2 * V]) {
  if (nv == V) {
    if constexpr (V == 1) {
      const float2 t = in[idx];
      v[0] = t.x;
      v[1] = t.y;
    } else {
#pragma unroll
      for (int h = 0; h < V / 2; ++h) {
        const float4_t t = *reinterpret_cast<const float4_t*>(in + idx + 2 * h);
        v[4 * h] = t[0];
        v[4 * h + 1] = t[1];
        v[4 * h + 2] = t[2];
        v[4 * h + 3] = t[3];
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) {
      float2 t = make_float2(0.f, 0.f);
      if (i < nv) t = in[idx + i];
      v[2 * i] = t.x;
      v[2 * i + 1] = t.y;
    }
  }
}

// PIPE: stage channel chunks through registers, prefetching chunk c + 1 from
// global memory while chunk c is multiplied (used when several chunks are
// streamed and a chunk fits in kStageSlots complex values per thread).
constexpr int kStageSlots = 16;

// Operand fragments of one k-block for one wave: FM row fragments from LDS,
// FN column fragments of the weights (L1/L2), hi and (split precision) lo.
template <int PREC, int FM, int FN> struct Frags;
template <int FM, int FN> struct Frags<P_F32, FM, FN> {
  float4_t a[FM], b[FN];
};
template <int FM, int FN> struct Frags<P_BF16, FM, FN> {
  bf16x8_t a[FM], b[FN];
};
template <int FM, int FN> struct Frags<P_BF16X3, FM, FN> {
  bf16x8_t a[FM], b[FN], al[FM], bl[FN];
};

// Stage channels [cbase, cbase + chunk_c) of the halo of one tile into LDS,
// V channels of one point per unit.  Units form a grid of rows (hh0, hh1)
// by columns (hh2, channel group); when a row of units fits the 256 threads
// each thread keeps its column (and that column's index arithmetic) and
// steps over rows, else units are enumerated one by one.
template <int PREC, int V>
__device__ __forceinline__ void stage_units(const ConvArgs& a, typename LdsElem<PREC>::T* lds,
                                            typename LdsElem<PREC>::T* lds_lo, const int cbase, const int64_t base0,
                                            const int64_t base1, const int64_t base2, const int tid) {
  const int cpr = a.chunk_c / V;
  const int ncol = a.h[2] * cpr;
  const int rows = a.h[0] * a.h[1];
  const int coff = cbase - a.chan_base;
  auto unit = [&](const int hh0, const int hh1, const int hh2, const int cq) {
    const int64_t i0 = a.org[0] + base0 + hh0, i1 = a.org[1] + base1 + hh1, i2 = a.org[2] + base2 + hh2;
    const bool ok = i0 >= a.vlo[0] && i0 < a.vhi[0] && i1 >= a.vlo[1] && i1 < a.vhi[1] && i2 >= a.vlo[2] &&
                    i2 < a.vhi[2];
    const int nv = ok ? max(0, min(V, a.cin - (cbase + cq * V))) : 0;
    float v[2 * V];
    load_unit<V>(a.in, nv ? i0 * a.is[0] + i1 * a.is[1] + i2 * a.is[2] + coff + cq * V : 0, nv, v);
    stage_store<PREC, V>(lds, lds_lo, (hh0 * a.h[1] + hh1) * a.rs + hh2 * a.ps + 2 * cq * V, v);
  };
  if (ncol <= 256) {
    const int R = 256 / ncol;
    const int r0 = tid / ncol, col = tid - r0 * ncol;
    if (r0 >= R) return;
    const int hh2 = col / cpr, cq = col - hh2 * cpr;
    int hh0 = r0 / a.h[1], hh1 = r0 - hh0 * a.h[1];
    for (int row = r0; row < rows; row += R) {
      unit(hh0, hh1, hh2, cq);
      hh1 += R;
      while (hh1 >= a.h[1]) {
        hh1 -= a.h[1];
        ++hh0;
      }
    }
  } else {
    for (int e = tid; e < rows * ncol; e += 256) {
      const int row = e / ncol, col = e - row * ncol;
      const int hh0 = row / a.h[1], hh1 = row - hh0 * a.h[1];
      const int hh2 = col / cpr, cq = col - hh2 * cpr;
      unit(hh0, hh1, hh2, cq);
    }
  }
}

// One output tile: position tile bx (of gx) and column block by.  Shared by
// the per-problem kernel and the persistent batched kernel.
template <int PREC, int T0, int T2, int WC, int FN, int D, bool PIPE>
__device__ __forceinline__ void conv_tile(const ConvArgs& a, const int64_t bx, const int by, const int64_t gx,
                                          unsigned char* smem) {
  constexpr int KB = kblock_of(PREC);
  constexpr int NFRAG = T0 * T2;
  constexpr int WR = 4 / WC;
  static_assert(4 % WC == 0 && NFRAG % WR == 0, "tile must give each wave whole fragments");
  constexpr int FM = NFRAG / WR;
  constexpr int BC = 16 * WC * FN;
  constexpr bool SPLIT = PREC == P_BF16X3;
  using E = typename LdsElem<PREC>::T;

  E* lds = reinterpret_cast<E*>(smem);
  const int lds_elems = a.h[0] * a.h[1] * a.rs;
  E* lds_lo = lds + lds_elems;

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, m = lane & 15;
  const int wr = wave / WC, wc = wave % WC;
  const int64_t t2i = bx % a.nt[2];
  const int64_t t1i = (bx / a.nt[2]) % a.nt[1];
  const int64_t t0i = bx / (a.nt[2] * a.nt[1]);
  const int64_t base0 = t0i * T0, base1 = t1i * 16, base2 = t2i * (T2 * D);
  const int n0w = a.col0 + by * BC + wc * 16 * FN;  // first weight column of this wave

  // Row tails and the padding of each point past its 2 chunk_c entries are
  // read with zero weights and must hold finite values.
  {
    const int tail = a.rs - a.h[2] * a.ps;
    const int nrows = a.h[0] * a.h[1];
    for (int e = tid; e < nrows * tail; e += 256) {
      const int off = (e / tail) * a.rs + a.h[2] * a.ps + (e % tail);
      lds[off] = E(0);
      if constexpr (SPLIT) lds_lo[off] = E(0);
    }
    const int pad = a.ps - 2 * a.chunk_c;
    if (pad > 0) {
      const int npts = nrows * a.h[2];
      for (int e = tid; e < npts * pad; e += 256) {
        const int pt = e / pad, r = pt / a.h[2];
        const int off = r * a.rs + (pt - r * a.h[2]) * a.ps + 2 * a.chunk_c + (e - pt * pad);
        lds[off] = E(0);
        if constexpr (SPLIT) lds_lo[off] = E(0);
      }
    }
  }

  float4_t acc[FM][FN];
#pragma unroll
  for (int f = 0; f < FM; ++f)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[f][j] = float4_t{0.f, 0.f, 0.f, 0.f};

  // Per-fragment LDS offsets of this lane's operand (without kernel shift).
  int frag_off[FM];
#pragma unroll
  for (int f = 0; f < FM; ++f) {
    const int fg = wr * FM + f;
    const int fa = fg / T2, fc = fg % T2;
    frag_off[f] = (fa * a.h[1] + m) * a.rs + fc * D * a.ps + g * (KB / 4);
  }

  const int half_ps = a.ps >> 1;
  const int npts_halo = a.h[0] * a.h[1] * a.h[2];
  const int nstage = npts_halo * half_ps;
  const int nkb = a.nkb, nk1 = a.k[1];
  const int total = a.k[0] * nk1 * nkb;

  // Operands of flattened k-step i = ((k0 * k1n) + k1) * nkb + t of chunk chg.
  auto load_frags = [&](Frags<PREC, FM, FN>& fr, const int chg, const int i) {
    const int kk = i / nkb, t = i - kk * nkb;
    const int k0 = kk / nk1, k1 = kk - k0 * nk1;
    const int shift = (k0 * a.h[1] + k1) * a.rs + t * KB;
    const size_t wt = ((((size_t)chg * a.k[0] + k0) * nk1 + k1) * nkb + t) * a.ncolp * KB +
                      (size_t)(n0w + m) * KB + g * (KB / 4);
    if constexpr (PREC == P_F32) {
      const float* Bp = reinterpret_cast<const float*>(a.B);
#pragma unroll
      for (int f = 0; f < FM; ++f) fr.a[f] = *reinterpret_cast<const float4_t*>(lds + frag_off[f] + shift);
#pragma unroll
      for (int j = 0; j < FN; ++j) fr.b[j] = *reinterpret_cast<const float4_t*>(Bp + wt + (size_t)j * 16 * KB);
    } else {
      const uint16_t* Bp = reinterpret_cast<const uint16_t*>(a.B);
#pragma unroll
      for (int f = 0; f < FM; ++f)
        fr.a[f] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(lds + frag_off[f] + shift));
#pragma unroll
      for (int j = 0; j < FN; ++j)
        fr.b[j] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(Bp + wt + (size_t)j * 16 * KB));
      if constexpr (SPLIT) {
        const uint16_t* Bl = reinterpret_cast<const uint16_t*>(a.Blo);
#pragma unroll
        for (int f = 0; f < FM; ++f)
          fr.al[f] =
              __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(lds_lo + frag_off[f] + shift));
#pragma unroll
        for (int j = 0; j < FN; ++j)
          fr.bl[j] =
              __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(Bl + wt + (size_t)j * 16 * KB));
      }
    }
  };
  auto mma = [&](const Frags<PREC, FM, FN>& fr) {
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        if constexpr (PREC == P_F32) {
          acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[f][0], fr.b[j][0], acc[f][j], 0, 0, 0);
          acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[f][1], fr.b[j][1], acc[f][j], 0, 0, 0);
          acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[f][2], fr.b[j][2], acc[f][j], 0, 0, 0);
          acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fr.a[f][3], fr.b[j][3], acc[f][j], 0, 0, 0);
        } else {
          acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr.a[f], fr.b[j], acc[f][j], 0, 0, 0);
          if constexpr (SPLIT) {
            acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr.a[f], fr.bl[j], acc[f][j], 0, 0, 0);
            acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr.al[f], fr.b[j], acc[f][j], 0, 0, 0);
          }
        }
      }
  };
  // The operands of step i + 1 are fetched while step i multiplies.
  auto compute_chunk = [&](const int chg) {
    Frags<PREC, FM, FN> p0, p1;
    load_frags(p0, chg, 0);
    for (int i = 0; i < total; i += 2) {
      if (i + 1 < total) load_frags(p1, chg, i + 1);
      mma(p0);
      if (i + 1 >= total) break;
      if (i + 2 < total) load_frags(p0, chg, i + 2);
      mma(p1);
    }
  };

  if constexpr (!PIPE) {
    for (int ch = 0; ch < a.nchunks; ++ch) {
      const int chg = a.ch0 + ch;
      __syncthreads();
      if (a.vec == 4) stage_units<PREC, 4>(a, lds, lds_lo, chg * a.chunk_c, base0, base1, base2, tid);
      else if (a.vec == 2) stage_units<PREC, 2>(a, lds, lds_lo, chg * a.chunk_c, base0, base1, base2, tid);
      else stage_units<PREC, 1>(a, lds, lds_lo, chg * a.chunk_c, base0, base1, base2, tid);
      __syncthreads();
      compute_chunk(chg);
    }
  } else {
    // Slot i of this thread stages complex value e = tid + 256 i of the
    // chunk: its point's input offset (or -1 outside the validity box), its
    // LDS offset and its channel slot, computed once for all chunks.
    int64_t goff[kStageSlots];
    int loff[kStageSlots], csl[kStageSlots];
#pragma unroll
    for (int i = 0; i < kStageSlots; ++i) {
      const int e = tid + 256 * i;
      goff[i] = -2;
      loff[i] = 0;
      csl[i] = 0;
      if (e < nstage) {
        const int cs = e % half_ps;
        const int pt = e / half_ps;
        const int hh2 = pt % a.h[2];
        const int q = pt / a.h[2];
        const int hh1 = q % a.h[1];
        const int hh0 = q / a.h[1];
        const int64_t i0 = a.org[0] + base0 + hh0;
        const int64_t i1 = a.org[1] + base1 + hh1;
        const int64_t i2 = a.org[2] + base2 + hh2;
        const bool ok = i0 >= a.vlo[0] && i0 < a.vhi[0] && i1 >= a.vlo[1] && i1 < a.vhi[1] && i2 >= a.vlo[2] &&
                        i2 < a.vhi[2];
        goff[i] = ok ? i0 * a.is[0] + i1 * a.is[1] + i2 * a.is[2] : -1;
        loff[i] = (hh0 * a.h[1] + hh1) * a.rs + hh2 * a.ps + 2 * cs;
        csl[i] = cs;
      }
    }
    float2 buf[kStageSlots];
    auto load = [&](const int chg) {
      const int cbase = chg * a.chunk_c;
#pragma unroll
      for (int i = 0; i < kStageSlots; ++i) {
        float2 v = make_float2(0.f, 0.f);
        if (goff[i] >= 0 && csl[i] < a.chunk_c && cbase + csl[i] < a.cin)
          v = a.in[goff[i] + (cbase - a.chan_base) + csl[i]];
        buf[i] = v;
      }
    };
    auto store = [&]() {
#pragma unroll
      for (int i = 0; i < kStageSlots; ++i)
        if (goff[i] != -2) {
          const float v[2] = {buf[i].x, buf[i].y};
          stage_store<PREC, 1>(lds, lds_lo, loff[i], v);
        }
    };
    load(a.ch0);
    __syncthreads();  // row tails zeroed before the first chunk lands
    store();
    __syncthreads();
    for (int ch = 0; ch < a.nchunks; ++ch) {
      const bool more = ch + 1 < a.nchunks;
      if (more) load(a.ch0 + ch + 1);
      compute_chunk(a.ch0 + ch);
      if (more) {
        __syncthreads();
        store();
        __syncthreads();
      }
    }
  }

  // Epilogue: lane holds rows 4g..4g+3 (positions along axis 1) of column m
  // of each of its FM x FN tiles.  Launch column lc = delta * coutr + c.
  double ssq = 0.0;
#pragma unroll
  for (int f = 0; f < FM; ++f) {
    const int fg = wr * FM + f;
    const int64_t p0 = base0 + fg / T2, p2b = base2 + (int64_t)(fg % T2) * D;
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int lc = by * BC + (wc * FN + j) * 16 + m;
      if (lc >= D * a.coutr) continue;
      const int delta = D == 1 ? 0 : lc / a.coutr;
      const int c = lc - delta * a.coutr;
      const int64_t p2 = p2b + delta;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t p1 = base1 + 4 * g + i;
        const bool pv = p0 < a.oe[0] && p1 < a.oe[1] && p2 < a.oe[2];
        if (!pv) continue;
        bool masked = false;
        if (a.mask)
          masked =
              a.mask[(a.morg[0] + p0) * a.ms[0] + (a.morg[1] + p1) * a.ms[1] + (a.morg[2] + p2) * a.ms[2]] != 0;
        float v = masked ? 0.f : acc[f][j][i] * a.scale;
        if (a.out) {
          float* dst = a.out + 2 * (p0 * a.os[0] + p1 * a.os[1] + p2 * a.os[2]) + c;
          if (a.accumulate) v += *dst;
          *dst = v;
        }
        ssq += (double)v * (double)v;
      }
    }
  }
  if (a.partial) {
    __shared__ double red[4];
    const double tot = block_sum_d(ssq, red);
    if (tid == 0) a.partial[(size_t)by * gx + bx] = tot;
  }
}

// Workgroups are dispatched to the 8 XCDs round-robin; remap the linear id so
// that each XCD (own L2) processes a contiguous run of work items: the
// column blocks of one position tile and neighbouring tiles along axis 2
// then share staged input through the same L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t w, int64_t W) {
  const int64_t per = W / 8, rem = W % 8;
  const int64_t xcd = w % 8, idx = w / 8;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

template <int PREC, int T0, int T2, int WC, int FN, int D, bool PIPE>
__global__ __launch_bounds__(256) void conv_kernel(ConvArgs a, int64_t gx, int gy) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t lin = xcd_remap(blockIdx.x, gx * gy);
  conv_tile<PREC, T0, T2, WC, FN, D, PIPE>(a, lin / gy, (int)(lin % gy), gx, smem);
}

// Persistent batched launch: the work list is every (position tile, column
// block) of every problem; tile_start[q] is the first work item of problem
// q.  Workgroups stride over the list, so problems of any size and channel
// count share one launch.  Each item runs the same tile code as the
// per-problem kernel, so results are bitwise identical.
template <int PREC, int T0, int T2, int WC, int FN, int D, bool PIPE>
__global__ __launch_bounds__(256) void conv_batch_kernel(const ConvArgs* args, const int64_t* tile_start, int nprob,
                                                         int64_t total) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tile_start[mid] <= it) lo = mid;
      else hi = mid - 1;
    }
    const ConvArgs& a = args[lo];
    const int64_t local = it - tile_start[lo];
    const int64_t gx = a.nt[0] * a.nt[1] * a.nt[2];
    conv_tile<PREC, T0, T2, WC, FN, D, PIPE>(a, local % gx, (int)(local / gx), gx, smem);
    __syncthreads();  // the next item reuses LDS
  }
}

// ---------------------------------------------------------------------------
// Weight builder
// ---------------------------------------------------------------------------
__device__ __forceinline__ void prep_element(const PrepArgs& a, const int64_t e) {
  const int kbe = (int)(e % a.KB);
  int64_t r = e / a.KB;
  const int col = (int)(r % a.ncolp);
  r /= a.ncolp;
  const int t = (int)(r % a.nkb);
  r /= a.nkb;
  const int k1 = (int)(r % a.k1);
  r /= a.k1;
  const int k0 = (int)(r % a.k0);
  const int ch = (int)(r / a.k0);
  const int run = t * a.KB + kbe;
  // launch column col = delta * coutr_total + c uses the taps shifted by delta
  const int delta = col / a.coutr_total, c = col - delta * a.coutr_total;
  const int kk2 = run / a.ps - delta, el = run % a.ps;
  float v = 0.f;
  if (delta < a.D && kk2 >= 0 && kk2 < a.k2 && el < 2 * a.chunk_c) {
    const int ci = ch * a.chunk_c + (el >> 1), ri = el & 1;
    const int co = c >> 1, ro = c & 1;
    if (a.mode == 0) {
      if (ci < a.nc && co < a.p) {
        const int64_t row = (((int64_t)k0 * a.k1 + k1) * a.k2 + kk2) * a.nc + ci;
        const float2 f = a.F[row * a.p + co];
        // y = x * f:  y.re = x.re f.re - x.im f.im,  y.im = x.re f.im + x.im f.re
        v = ri == 0 ? (ro == 0 ? f.x : f.y) : (ro == 0 ? -f.y : f.x);
      }
    } else {
      if (ci < a.p && co < a.nc) {
        const int64_t row = ((((int64_t)a.k0 - 1 - k0) * a.k1 + (a.k1 - 1 - k1)) * a.k2 + (a.k2 - 1 - kk2)) * a.nc + co;
        const float2 f = a.F[row * a.p + ci];
        // z = y * conj(f): z.re = y.re f.re + y.im f.im,  z.im = y.im f.re - y.re f.im
        v = ri == 0 ? (ro == 0 ? f.x : -f.y) : (ro == 0 ? f.y : f.x);
      }
    }
  }
  if (a.prec == P_F32) {
    reinterpret_cast<float*>(a.B)[e] = v;
  } else {
    const uint16_t h = f2bf(v);
    reinterpret_cast<uint16_t*>(a.B)[e] = h;
    if (a.prec == P_BF16X3) reinterpret_cast<uint16_t*>(a.Blo)[e] = f2bf(v - bf2f(h));
  }
}

__global__ void prep_weights_kernel(PrepArgs a) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.total;
       e += (int64_t)gridDim.x * blockDim.x)
    prep_element(a, e);
}

// Batched weight builder: blockIdx.y selects the problem.
__global__ void prep_weights_batch_kernel(const PrepArgs* args) {
  const PrepArgs& a = args[blockIdx.y];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.total;
       e += (int64_t)gridDim.x * blockDim.x)
    prep_element(a, e);
}

__global__ __launch_bounds__(1024) void reduce_kernel(const double* part, int64_t count, double* out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += blockDim.x) s += part[i];
  const double tot = block_sum_d(s, red);
  if (threadIdx.x == 0) *out = tot;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
TileCfg tile_cfg(int id) {
  static const TileCfg table[kNumTiles] = {
#define HICU_TILE_ROW(id, T0, T2, WC, FN, D, P, B) {T0, T2, WC, FN, D},
      HICU_TILES(HICU_TILE_ROW)
#undef HICU_TILE_ROW
  };
  return (id >= 0 && id < kNumTiles) ? table[id] : TileCfg{0, 0, 0, 0, 0};
}

static bool tile_pipe_ok(int id) {
  static const bool table[kNumTiles] = {
#define HICU_TILE_ROW(id, T0, T2, WC, FN, D, P, B) P != 0,
      HICU_TILES(HICU_TILE_ROW)
#undef HICU_TILE_ROW
  };
  return id >= 0 && id < kNumTiles && table[id];
}

WeightShape weight_shape(int prec, const int k[3], int cin, int chunk_c, int coutr_total, int D) {
  WeightShape w;
  w.KB = kblock_of(prec);
  w.D = D;
  w.cout = coutr_total;
  w.chunk_c = chunk_c;
  w.nchunks = (int)cdiv(cin, chunk_c);
  w.ps = (int)rup(2 * chunk_c, 8);
  w.nkb = (int)cdiv((int64_t)(k[2] + D - 1) * w.ps, w.KB);
  w.ncolp = (int)rup((int64_t)D * coutr_total, kColPad);
  w.elems = (size_t)w.nchunks * k[0] * k[1] * w.nkb * w.ncolp * w.KB;
  return w;
}

PrepArgs make_prep_args(int mode, int prec, const Geo& g, const float2* F, int p, const WeightShape& ws, void* B,
                        void* Blo) {
  PrepArgs a;
  a.F = F;
  a.p = p;
  a.nc = g.nc;
  a.k0 = g.k[0];
  a.k1 = g.k[1];
  a.k2 = g.k[2];
  a.mode = mode;
  a.prec = prec;
  a.chunk_c = ws.chunk_c;
  a.ps = ws.ps;
  a.nkb = ws.nkb;
  a.ncolp = ws.ncolp;
  a.KB = ws.KB;
  a.coutr_total = mode == 0 ? 2 * p : 2 * g.nc;
  a.D = ws.D;
  a.total = (int64_t)ws.elems;
  a.B = B;
  a.Blo = Blo;
  return a;
}

int32_t launch_prep_weights(int mode, int prec, const Geo& g, const float2* F, int p,
                            const WeightShape& ws, void* B, void* Blo, hipStream_t st) {
  const PrepArgs a = make_prep_args(mode, prec, g, F, p, ws, B, Blo);
  if (ws.cout != a.coutr_total) return HICU_ERR_SHAPE;
  const int64_t blocks = std::min<int64_t>(cdiv(a.total, 256), 8192);
  hipLaunchKernelGGL(prep_weights_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

int32_t launch_prep_weights_batch(const PrepArgs* args_dev, int count, int64_t max_total, hipStream_t st) {
  if (count < 1 || count > 65535) return HICU_ERR_ARG;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(max_total, 256), 2048));
  hipLaunchKernelGGL(prep_weights_batch_kernel, dim3((unsigned)blocks, (unsigned)count), dim3(256), 0, st, args_dev);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

static int64_t stage_elems(const ConvPlan& p) {
  return (int64_t)p.a.h[0] * p.a.h[1] * p.a.h[2] * (p.a.ps / 2);
}

bool conv_can_pipe(const ConvPlan& p) { return tile_pipe_ok(p.tile) && stage_elems(p) <= 256 * kStageSlots; }

int conv_vec(const ConvArgs& a) {
  const bool aligned = (reinterpret_cast<uintptr_t>(a.in) & 15) == 0;
  for (int V : {4, 2}) {
    if (aligned && a.is[2] % V == 0 && a.chunk_c % V == 0 && a.chan_base % V == 0) return V;
  }
  return 1;
}

// Per-problem launches: one 1-D grid of gx * gy workgroups.
template <int PREC>
static int32_t launch_prec(const ConvPlan& p, bool pipe, hipStream_t st) {
  const dim3 grid((unsigned)(p.gx * p.gy)), block(256);
  switch (p.tile) {
#define HICU_TILE_CASE(id, T0, T2, WC, FN, D, P, B)                                                              \
  case id:                                                                                                     \
    if constexpr (P != 0) {                                                                                    \
      if (pipe) {                                                                                              \
        hipLaunchKernelGGL((conv_kernel<PREC, T0, T2, WC, FN, D, true>), grid, block, p.lds_bytes, st, p.a,     \
                           p.gx, p.gy);                                                                        \
        break;                                                                                                 \
      }                                                                                                        \
    }                                                                                                          \
    hipLaunchKernelGGL((conv_kernel<PREC, T0, T2, WC, FN, D, false>), grid, block, p.lds_bytes, st, p.a, p.gx,  \
                       p.gy);                                                                                  \
    break;
    HICU_TILES(HICU_TILE_CASE)
#undef HICU_TILE_CASE
    default:
      return HICU_ERR_UNSUPPORTED;
  }
  return HICU_OK;
}

template <int PREC>
static int32_t launch_batch_prec(const BatchConvLaunch& b, hipStream_t st) {
  const dim3 grid(b.grid), block(256);
  switch (b.tile) {
#define HICU_TILE_CASE(id, T0, T2, WC, FN, D, P, B)                                                            \
  case id:                                                                                                   \
    if constexpr (B != 0) {                                                                                  \
      if (b.pipe)                                                                                            \
        hipLaunchKernelGGL((conv_batch_kernel<PREC, T0, T2, WC, FN, D, true>), grid, block, b.lds_bytes, st,  \
                           b.args, b.tile_start, b.nprob, b.total);                                          \
      else                                                                                                   \
        hipLaunchKernelGGL((conv_batch_kernel<PREC, T0, T2, WC, FN, D, false>), grid, block, b.lds_bytes, st, \
                           b.args, b.tile_start, b.nprob, b.total);                                          \
      break;                                                                                                 \
    }                                                                                                        \
    return HICU_ERR_UNSUPPORTED;
    HICU_TILES(HICU_TILE_CASE)
#undef HICU_TILE_CASE
    default:
      return HICU_ERR_UNSUPPORTED;
  }
  return HICU_OK;
}

int32_t launch_conv_batch(const BatchConvLaunch& b, hipStream_t st) {
  if (b.nprob < 1 || b.total < 1 || b.grid < 1) return HICU_ERR_ARG;
  if (b.lds_bytes > kMaxLds) return HICU_ERR_UNSUPPORTED;
  int32_t s;
  if (b.prec == P_F32) s = launch_batch_prec<P_F32>(b, st);
  else if (b.prec == P_BF16) s = launch_batch_prec<P_BF16>(b, st);
  else s = launch_batch_prec<P_BF16X3>(b, st);
  if (s != HICU_OK) return s;
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

// Shapes tried first: the widest column block the output fills, D > 1 for
// narrow outputs when the kernel has at least 3 taps along axis 2 (the
// packing lengthens the reduction by (k2 + D - 1) / k2).
int default_tile(int prec, const Geo& g, int coutr, int role) {
  (void)prec;
  const bool is3d = g.k[0] > 1;
  const int frags = (int)cdiv(coutr, 16);
  if (role == 1 && g.k[2] >= 3 && frags <= 2) {
    if (frags == 1) return is3d ? 21 : 12;
    return is3d ? 24 : 10;
  }
  if (frags >= 8) return is3d ? 19 : 7;
  if (frags >= 3) return is3d ? 15 : 2;
  if (frags == 2) return is3d ? 14 : 1;
  return is3d ? 13 : 0;
}

static int pick_rs(int prec, int need) {
  if (prec == P_F32) {
    int rs = (int)rup(need, 4);
    while (rs % 64 != 4) rs += 4;
    return rs;
  }
  int rs = (int)rup(need, 8);
  while (rs % 128 != 8) rs += 8;
  return rs;
}

int32_t plan_conv(int prec, int tile, const int k[3], const WeightShape& ws, int nchunks,
                  const int64_t oe[3], int coutr, ConvPlan* plan) {
  const TileCfg t = tile_cfg(tile);
  if (t.T0 < 1) return HICU_ERR_ARG;
  if (ws.D != t.D) return HICU_ERR_ARG;
  ConvArgs& a = plan->a;
  plan->prec = prec;
  plan->tile = tile;
  plan->t = t;
  a.chunk_c = ws.chunk_c;
  a.chan_base = 0;
  a.nchunks = nchunks;
  a.ps = ws.ps;
  a.nkb = ws.nkb;
  a.ncolp = ws.ncolp;
  for (int i = 0; i < 3; ++i) a.k[i] = k[i];
  a.h[0] = t.T0 + k[0] - 1;
  a.h[1] = 16 + k[1] - 1;
  a.h[2] = t.T2 * t.D + k[2] - 1;
  const int need = (t.T2 - 1) * t.D * ws.ps + ws.nkb * ws.KB;
  a.rs = pick_rs(prec, need);
  const size_t esize = prec == P_F32 ? 4 : 2;
  plan->lds_bytes = (size_t)a.h[0] * a.h[1] * a.rs * esize * (prec == P_BF16X3 ? 2 : 1);
  if (plan->lds_bytes > kMaxLds) return HICU_ERR_UNSUPPORTED;
  a.oe[0] = oe[0];
  a.oe[1] = oe[1];
  a.oe[2] = oe[2];
  a.nt[0] = cdiv(oe[0], t.T0);
  a.nt[1] = cdiv(oe[1], 16);
  a.nt[2] = cdiv(oe[2], (int64_t)t.T2 * t.D);
  const int64_t gx = a.nt[0] * a.nt[1] * a.nt[2];
  const int64_t gy = cdiv((int64_t)t.D * coutr, block_cols(t));
  if (gx <= 0 || gy <= 0 || gy > 65535 || gx * gy > 0x7fffffff) return HICU_ERR_SHAPE;
  a.coutr = coutr;
  plan->gx = gx;
  plan->gy = (int)gy;
  return HICU_OK;
}

int32_t launch_conv(const ConvPlan& p, hipStream_t st) {
  // Host-side guard of every index the kernel forms from its arguments.
  const ConvArgs& a = p.a;
  const TileCfg t = tile_cfg(p.tile);
  if (t.T0 < 1 || t.D != p.t.D) return HICU_ERR_ARG;
  if ((int64_t)a.col0 + (int64_t)p.gy * block_cols(t) > a.ncolp) return HICU_ERR_SHAPE;
  if ((int64_t)p.gy * block_cols(t) < (int64_t)t.D * a.coutr) return HICU_ERR_SHAPE;
  if (a.ps < 2 * a.chunk_c || a.ps % 8 != 0) return HICU_ERR_SHAPE;
  if (a.rs < (t.T2 - 1) * t.D * a.ps + a.nkb * kblock_of(p.prec)) return HICU_ERR_SHAPE;
  if (a.nkb * kblock_of(p.prec) < (a.k[2] + t.D - 1) * a.ps) return HICU_ERR_SHAPE;
  if (a.h[2] != t.T2 * t.D + a.k[2] - 1 || a.h[1] != 16 + a.k[1] - 1 || a.h[0] != t.T0 + a.k[0] - 1)
    return HICU_ERR_SHAPE;
  if ((int64_t)a.ch0 * a.chunk_c < a.chan_base) return HICU_ERR_SHAPE;
  if (p.lds_bytes > kMaxLds || p.gx * p.gy > 0x7fffffff) return HICU_ERR_SHAPE;
  const bool pipe = a.nchunks > 1 && conv_can_pipe(p);
  ConvPlan q = p;
  q.a.vec = conv_vec(a);
  int32_t s;
  if (p.prec == P_F32) s = launch_prec<P_F32>(q, pipe, st);
  else if (p.prec == P_BF16) s = launch_prec<P_BF16>(q, pipe, st);
  else s = launch_prec<P_BF16X3>(q, pipe, st);
  if (s != HICU_OK) return s;
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

int32_t launch_reduce(const double* part, int64_t count, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, part, count, out);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

}  // namespace hicu
