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
#pragma once

#include <algorithm>

#include "conv.h"

namespace hicu {

template <int PREC> struct LdsElem { using T = float; };
template <> struct LdsElem<P_BF16> { using T = uint16_t; };
template <> struct LdsElem<P_BF16X3> { using T = uint16_t; };
template <> struct LdsElem<P_F16> { using T = uint16_t; };

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

typedef float float2v_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));

// Two floats -> packed BF16 (round to nearest even; one v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t pack_bf16(float x, float y) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(float2v_t{x, y}, bf16x2_t));
}
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
// Two floats -> packed FP16 (round to nearest even; one v_cvt_pk_f16_f32).
__device__ __forceinline__ uint32_t pack_f16(float x, float y) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(float2v_t{x, y}, f16x2_t));
}
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// Store 2V floats (V complex values, interleaved re/im) at LDS element
// offset off: FP32 as is, BF16 rounded, split BF16 as hi and lo = v - hi.
template <int PREC, int V>
__device__ __forceinline__ void stage_store(typename LdsElem<PREC>::T* hi, typename LdsElem<PREC>::T* lo, int off,
                                            const float (&v)[2 * V], const float sc) {
  if constexpr (PREC == P_F16) {
    uint32_t w[V];
#pragma unroll
    for (int i = 0; i < V; ++i) w[i] = pack_f16(v[2 * i] * sc, v[2 * i + 1] * sc);
    if constexpr (V == 4) *reinterpret_cast<u32x4_t*>(hi + off) = u32x4_t{w[0], w[1], w[2], w[3]};
    else if constexpr (V == 2) *reinterpret_cast<u32x2_t*>(hi + off) = u32x2_t{w[0], w[1]};
    else *reinterpret_cast<uint32_t*>(hi + off) = w[0];
  } else if constexpr (PREC == P_F32) {
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
// Index on an axis of period P (0: not circular), for i within one period
// of [0, P); the result is then checked against the validity box.
__device__ __forceinline__ int64_t wrap_index(int64_t i, int64_t P) {
  if (P == 0) return i;
  return i < 0 ? i + P : (i >= P ? i - P : i);
}

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

// Operand fragments of one k-step for one wave: FM row fragments from LDS
// (FragA), FN column fragments of the weights from L1/L2 (FragB); hi and, for
// the split precision, lo parts.
template <int PREC, int FM> struct FragA {
  bf16x8_t a[FM];
};
template <int FM> struct FragA<P_F32, FM> {
  float4_t a[FM];
};
template <int FM> struct FragA<P_BF16X3, FM> {
  bf16x8_t a[FM], al[FM];
};
template <int FM> struct FragA<P_F16, FM> {
  f16x8_t a[FM];
};
template <int PREC, int FN> struct FragB {
  bf16x8_t b[FN];
};
template <int FN> struct FragB<P_F32, FN> {
  float4_t b[FN];
};
template <int FN> struct FragB<P_BF16X3, FN> {
  bf16x8_t b[FN], bl[FN];
};
template <int FN> struct FragB<P_F16, FN> {
  f16x8_t b[FN];
};

// Weight prefetch distance in k-steps (odd: the ring of PD + 1 register
// sets must be even).  A step issues FM * FN MFMAs; small register tiles
// look further ahead to cover the L2 latency, while the 4 x 4 tiles keep a
// one-step lookahead: a deeper ring costs them the second wave per SIMD
// (measured: 0.19 ms instead of 0.12 ms for the 256 x 232 x 16 forward).
template <int FM, int FN> constexpr int prefetch_distance() {
  return FM * FN >= 16 ? 1 : (FM * FN >= 8 ? 3 : 7);
}

// V BF16 (re, im) pairs from a compact residual at in + idx (nv < V: one by
// one, the rest zero).
template <int V>
__device__ __forceinline__ void load_unit_bf16(const uint32_t* in, int64_t idx, int nv, uint32_t (&w)[V]) {
  if (nv == V) {
    if constexpr (V == 4) {
      const u32x4_t t = *reinterpret_cast<const u32x4_t*>(in + idx);
      w[0] = t[0];
      w[1] = t[1];
      w[2] = t[2];
      w[3] = t[3];
    } else if constexpr (V == 2) {
      const u32x2_t t = *reinterpret_cast<const u32x2_t*>(in + idx);
      w[0] = t[0];
      w[1] = t[1];
    } else {
      w[0] = in[idx];
    }
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) w[i] = i < nv ? in[idx + i] : 0u;
  }
}

template <int V>
__device__ __forceinline__ void store_unit_bf16(uint16_t* lds, int off, const uint32_t (&w)[V]) {
  if constexpr (V == 4) *reinterpret_cast<u32x4_t*>(lds + off) = u32x4_t{w[0], w[1], w[2], w[3]};
  else if constexpr (V == 2) *reinterpret_cast<u32x2_t*>(lds + off) = u32x2_t{w[0], w[1]};
  else *reinterpret_cast<uint32_t*>(lds + off) = w[0];
}

// Stage channels [cbase, cbase + chunk_c) of the halo of one tile into LDS,
// V channels of one point per unit.  Units form a grid of rows (hh0, hh1)
// by columns (hh2, channel group); when a row of units fits the 256 threads
// each thread keeps its column (and that column's index arithmetic) and
// steps over rows, else units are enumerated one by one.  IB: the input is
// a compact BF16 residual, copied as it is; a thread then issues the loads
// of a batch of units (16 data registers' worth) before their LDS stores,
// so that many loads are in flight at once.  Complex64 input keeps one unit
// in flight: batching it raised the register count of the large tiles past
// the two waves per SIMD they run at.

template <int PREC, int V, bool IB = false>
__device__ __forceinline__ void stage_units(const ConvArgs& a, typename LdsElem<PREC>::T* lds,
                                            typename LdsElem<PREC>::T* lds_lo, const int cbase, const int64_t base0,
                                            const int64_t base1, const int64_t base2, const int tid, const float sc) {
  static_assert(!IB || PREC == P_BF16, "compact residual input is BF16");
  const int cpr = a.chunk_c / V;
  const int ncol = a.h[2] * cpr;
  const int rows = a.h[0] * a.h[1];
  // complex64 input: channel offset inside a point; compact BF16 input: the
  // chunk's block (a chunk is one block)
  const int64_t coff = IB ? (int64_t)((cbase - a.chan_base) / a.chunk_c) * a.yblk : (int64_t)(cbase - a.chan_base);
  constexpr int SB = IB ? 16 / V : 1;
  float fv[SB][2 * V];
  uint32_t wv[SB][V];
  int loff[SB];
  auto fetch = [&](const int b, const int hh0, const int hh1, const int hh2, const int cq) {
    const int64_t i0 = wrap_index(a.org[0] + base0 + hh0, a.wp[0]);
    const int64_t i1 = wrap_index(a.org[1] + base1 + hh1, a.wp[1]);
    const int64_t i2 = wrap_index(a.org[2] + base2 + hh2, a.wp[2]);
    const bool ok = i0 >= a.vlo[0] && i0 < a.vhi[0] && i1 >= a.vlo[1] && i1 < a.vhi[1] && i2 >= a.vlo[2] &&
                    i2 < a.vhi[2];
    const int nv = ok ? max(0, min(V, a.cin - (cbase + cq * V))) : 0;
    const int64_t idx = nv ? i0 * a.is[0] + i1 * a.is[1] + i2 * a.is[2] + coff + cq * V : 0;
    loff[b] = (hh0 * a.h[1] + hh1) * a.rs + hh2 * a.ps + 2 * cq * V;
    if constexpr (IB) load_unit_bf16<V>(reinterpret_cast<const uint32_t*>(a.in), idx, nv, wv[b]);
    else load_unit<V>(a.in, idx, nv, fv[b]);
  };
  auto put = [&](const int b) {
    if constexpr (IB) store_unit_bf16<V>(lds, loff[b], wv[b]);
    else stage_store<PREC, V>(lds, lds_lo, loff[b], fv[b], sc);
  };
  if (ncol <= 256) {
    const int R = 256 / ncol;
    const int r0 = tid / ncol, col = tid - r0 * ncol;
    if (r0 >= R) return;
    const int hh2 = col / cpr, cq = col - hh2 * cpr;
    int hh0 = r0 / a.h[1], hh1 = r0 - hh0 * a.h[1];
    for (int row = r0; row < rows; row += SB * R) {
      int nb = 0;
#pragma unroll
      for (int b = 0; b < SB; ++b) {
        if (row + b * R < rows) {
          fetch(b, hh0, hh1, hh2, cq);
          nb = b + 1;
          hh1 += R;
          while (hh1 >= a.h[1]) {
            hh1 -= a.h[1];
            ++hh0;
          }
        }
      }
#pragma unroll
      for (int b = 0; b < SB; ++b)
        if (b < nb) put(b);
    }
  } else {
    const int total = rows * ncol;
    for (int e0 = tid; e0 < total; e0 += SB * 256) {
      int nb = 0;
#pragma unroll
      for (int b = 0; b < SB; ++b) {
        const int e = e0 + b * 256;
        if (e < total) {
          const int row = e / ncol, col = e - row * ncol;
          const int hh0 = row / a.h[1], hh1 = row - hh0 * a.h[1];
          const int hh2 = col / cpr, cq = col - hh2 * cpr;
          fetch(b, hh0, hh1, hh2, cq);
          nb = b + 1;
        }
      }
#pragma unroll
      for (int b = 0; b < SB; ++b)
        if (b < nb) put(b);
    }
  }
}

// One output tile: position tile bx (of gx) and column block by.  Shared by
// the per-problem kernel and the persistent batched kernel.
template <int PREC, int T0, int T2, int WC, int FN, int D, int KS, bool PIPE, int YB = 0>
__device__ __forceinline__ void conv_tile(const ConvArgs& a, const int64_t bx, const int by, const int64_t gx,
                                          unsigned char* smem) {
  static_assert(YB == 0 || (PREC == P_BF16 && !PIPE), "compact residual: BF16, unpipelined");
  constexpr int KB = kblock_of(PREC);
  constexpr int NFRAG = T0 * T2;
  constexpr int WR = 4 / (WC * KS);
  static_assert(4 % (WC * KS) == 0 && NFRAG % WR == 0, "tile must give each wave whole fragments");
  constexpr int FM = NFRAG / WR;
  static_assert(FM % KS == 0, "a k-split's epilogue gives each wave whole fragments");
  constexpr int FE = FM / KS;  // fragments of this wave in the epilogue
  constexpr int BC = 16 * WC * FN;
  constexpr bool SPLIT = PREC == P_BF16X3;
  using E = typename LdsElem<PREC>::T;

  E* lds = reinterpret_cast<E*>(smem);
  const int lds_elems = a.h[0] * a.h[1] * a.rs;
  E* lds_lo = lds + lds_elems;

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, m = lane & 15;
  // wave = (wr * WC + wc) * KS + ks: ks picks the k-steps of a k-split
  const int ks = wave % KS, wgrp = wave / KS, wr = wgrp / WC, wc = wgrp % WC;
  const int64_t t2i = bx % a.nt[2];
  const int64_t t1i = (bx / a.nt[2]) % a.nt[1];
  const int64_t t0i = bx / (a.nt[2] * a.nt[1]);
  const int64_t base0 = t0i * T0, base1 = t1i * 16, base2 = t2i * (T2 * D);
  const int n0w = a.col0 + by * BC + wc * 16 * FN;  // first weight column of this wave
  // Input scale (a power of two, FP16 only) and its exact inverse for the epilogue.
  const float in_sc = a.in_scale ? *a.in_scale : 1.f;
  const float out_sc = a.in_scale ? a.scale / in_sc : a.scale;

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
  const int nkb = a.nkb, nk1 = a.k[1];
  const int total = a.k[0] * nk1 * nkb;

  // Operands of k-step i = ((k0 * k1n) + k1) * nkb + t of a chunk.  The LDS
  // shift of a step is (k0 h1 + k1) rs + t KB and the weights of the steps
  // of chunk chg are consecutive rows of ncolp * KB elements, so both are
  // advanced incrementally (scalar adds) instead of being recomputed.
  using BE = typename LdsElem<PREC>::T;  // weight element type matches the LDS type
  auto load_a = [&](FragA<PREC, FM>& fr, const int shift) {
#pragma unroll
    for (int f = 0; f < FM; ++f) {
      if constexpr (PREC == P_F32) {
        fr.a[f] = *reinterpret_cast<const float4_t*>(lds + frag_off[f] + shift);
      } else if constexpr (PREC == P_F16) {
        fr.a[f] = __builtin_bit_cast(f16x8_t, *reinterpret_cast<const u32x4_t*>(lds + frag_off[f] + shift));
      } else {
        fr.a[f] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(lds + frag_off[f] + shift));
        if constexpr (SPLIT)
          fr.al[f] =
              __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(lds_lo + frag_off[f] + shift));
      }
    }
  };
  const uint32_t wlane = (uint32_t)((n0w + m) * KB + g * (KB / 4));
  const size_t wstep = (size_t)a.ncolp * KB;  // elements per k-step row
  auto load_b = [&](FragB<PREC, FN>& fr, const BE* bhi, const BE* blo) {
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      if constexpr (PREC == P_F32) {
        fr.b[j] = *reinterpret_cast<const float4_t*>(bhi + wlane + j * 16 * KB);
      } else if constexpr (PREC == P_F16) {
        fr.b[j] = __builtin_bit_cast(f16x8_t, *reinterpret_cast<const u32x4_t*>(bhi + wlane + j * 16 * KB));
      } else {
        fr.b[j] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(bhi + wlane + j * 16 * KB));
        if constexpr (SPLIT)
          fr.bl[j] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(blo + wlane + j * 16 * KB));
      }
    }
  };
  auto mma = [&](const FragA<PREC, FM>& fa, const FragB<PREC, FN>& fb) {
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        if constexpr (PREC == P_F32) {
          acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.a[f][0], fb.b[j][0], acc[f][j], 0, 0, 0);
          acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.a[f][1], fb.b[j][1], acc[f][j], 0, 0, 0);
          acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.a[f][2], fb.b[j][2], acc[f][j], 0, 0, 0);
          acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.a[f][3], fb.b[j][3], acc[f][j], 0, 0, 0);
        } else if constexpr (PREC == P_F16) {
          acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fa.a[f], fb.b[j], acc[f][j], 0, 0, 0);
        } else {
          acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa.a[f], fb.b[j], acc[f][j], 0, 0, 0);
          if constexpr (SPLIT) {
            acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa.a[f], fb.bl[j], acc[f][j], 0, 0, 0);
            acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa.al[f], fb.b[j], acc[f][j], 0, 0, 0);
          }
        }
      }
  };
  // Weights are fetched PD steps ahead into a ring of NB = PD + 1 register
  // sets, LDS operands one step ahead (double buffered); the loop is
  // unrolled by NB so every ring index is static.
  constexpr int PD = SPLIT ? 1 : prefetch_distance<FM, FN>();
  constexpr int NB = PD + 1;
  static_assert(NB % 2 == 0, "ring size must be even");
  // A wave whose columns all lie past the launch's last column (the tail
  // of the last column block) has nothing to accumulate: it skips the
  // k-loop (its accumulators stay zero and are never stored).
  const bool live_cols = by * BC + wc * FN * 16 < D * a.coutr;
  auto compute_chunk_flat = [&](const int chg) {
    if (!live_cols) return;
    FragA<PREC, FM> fa[2];
    FragB<PREC, FN> fb[NB];
    const BE* bhi0 = reinterpret_cast<const BE*>(a.B) + (size_t)chg * total * wstep;
    const BE* blo0 = reinterpret_cast<const BE*>(a.Blo) + (size_t)chg * total * wstep;
    // weights of step i (clamped to the last step: a redundant reload keeps
    // the main loop free of branches, so every wait counts only the loads
    // it needs)
    auto load_b_at = [&](FragB<PREC, FN>& fr, const int i) {
      const size_t o = (size_t)min(i, total - 1) * wstep;
      load_b(fr, bhi0 + o, blo0 + o);
    };
    int shift = 0, st = 0, sk1 = 0, left = total - 1;  // LDS shift of the next A step
    auto next_a = [&](FragA<PREC, FM>& fr) {
      load_a(fr, shift);
      if (left > 0) {  // uniform: advance unless the last step was loaded
        --left;
        shift += KB;
        if (++st == nkb) {
          st = 0;
          shift += a.rs - nkb * KB;
          if (++sk1 == nk1) {
            sk1 = 0;
            shift += (a.h[1] - nk1) * a.rs;
          }
        }
      }
    };
#pragma unroll
    for (int u = 0; u < PD; ++u) load_b_at(fb[u], u);
    next_a(fa[0]);
    int i0 = 0;
    for (; i0 + NB <= total; i0 += NB) {
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        load_b_at(fb[(u + PD) % NB], i0 + u + PD);
        next_a(fa[(u + 1) % 2]);
        mma(fa[u % 2], fb[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      if (i0 + u < total) {
        load_b_at(fb[(u + PD) % NB], i0 + u + PD);
        next_a(fa[(u + 1) % 2]);
        mma(fa[u % 2], fb[u]);
      }
    }
  };

  // Register-pipelined staging keeps the next chunk's halo loads in flight
  // during the MFMAs; the memory counter completes in order, so the precise
  // waits of the flat loop would also wait for those loads.  That variant
  // keeps per-step guards instead (measured faster for it).
  auto compute_chunk_guarded = [&](const int chg) {
    FragA<PREC, FM> fa[2];
    FragB<PREC, FN> fb[NB];
    const BE* bhi = reinterpret_cast<const BE*>(a.B) + (size_t)chg * total * wstep;
    const BE* blo = reinterpret_cast<const BE*>(a.Blo) + (size_t)chg * total * wstep;
    auto next_b = [&](FragB<PREC, FN>& fr) {
      load_b(fr, bhi, blo);
      bhi += wstep;
      blo += wstep;
    };
    int shift = 0, st = 0, sk1 = 0;
    auto next_a = [&](FragA<PREC, FM>& fr) {
      load_a(fr, shift);
      shift += KB;
      if (++st == nkb) {
        st = 0;
        shift += a.rs - nkb * KB;
        if (++sk1 == nk1) {
          sk1 = 0;
          shift += (a.h[1] - nk1) * a.rs;
        }
      }
    };
#pragma unroll
    for (int u = 0; u < PD; ++u)
      if (u < total) next_b(fb[u]);
    next_a(fa[0]);
    for (int i0 = 0; i0 < total; i0 += NB) {
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int i = i0 + u;
        if (i < total) {
          if (i + PD < total) next_b(fb[(u + PD) % NB]);
          if (i + 1 < total) next_a(fa[(u + 1) % 2]);
          mma(fa[u % 2], fb[u]);
        }
      }
    }
  };
  // Wave k-split: steps ks, ks + KS, ... of the chunk, operands one step
  // ahead (A and B double buffered); the step's LDS shift is formed from its
  // index (k0 h1 + k1) rs + t KB.
  auto compute_chunk_ks = [&](const int chg) {
    const BE* bhi0 = reinterpret_cast<const BE*>(a.B) + (size_t)chg * total * wstep;
    const BE* blo0 = reinterpret_cast<const BE*>(a.Blo) + (size_t)chg * total * wstep;
    auto shift_of = [&](const int i) {
      const int t = i % nkb, kk = i / nkb;
      return ((kk / nk1) * a.h[1] + kk % nk1) * a.rs + t * KB;
    };
    int i = ks;
    if (i >= total) return;
    FragA<PREC, FM> fa0, fa1;
    FragB<PREC, FN> fb0, fb1;
    load_b(fb0, bhi0 + (size_t)i * wstep, blo0 + (size_t)i * wstep);
    load_a(fa0, shift_of(i));
    for (;;) {
      const int i1 = i + KS;
      if (i1 < total) {
        load_b(fb1, bhi0 + (size_t)i1 * wstep, blo0 + (size_t)i1 * wstep);
        load_a(fa1, shift_of(i1));
      }
      mma(fa0, fb0);
      if (i1 >= total) break;
      const int i2 = i1 + KS;
      if (i2 < total) {
        load_b(fb0, bhi0 + (size_t)i2 * wstep, blo0 + (size_t)i2 * wstep);
        load_a(fa0, shift_of(i2));
      }
      mma(fa1, fb1);
      if (i2 >= total) break;
      i = i2;
    }
  };
  auto compute_chunk = [&](const int chg) {
    if constexpr (KS > 1) compute_chunk_ks(chg);
    else if constexpr (PIPE) compute_chunk_guarded(chg);
    else compute_chunk_flat(chg);
  };

  if constexpr (!PIPE) {
    for (int ch = 0; ch < a.nchunks; ++ch) {
      const int chg = a.ch0 + ch;
      __syncthreads();
      constexpr bool IB = YB == 1;
      if (a.vec == 4) stage_units<PREC, 4, IB>(a, lds, lds_lo, chg * a.chunk_c, base0, base1, base2, tid, in_sc);
      else if (a.vec == 2)
        stage_units<PREC, 2, IB>(a, lds, lds_lo, chg * a.chunk_c, base0, base1, base2, tid, in_sc);
      else stage_units<PREC, 1, IB>(a, lds, lds_lo, chg * a.chunk_c, base0, base1, base2, tid, in_sc);
      __syncthreads();
      compute_chunk(chg);
    }
  } else {
    // Slot i of this thread stages the group of VS = 4 consecutive channels
    // g = tid + 256 i of the chunk (pipelined launches require the input's
    // channel runs to be 16-byte aligned, a.vec == 4): its point's input
    // offset (or -1 outside the validity box), its LDS offset and its first
    // channel, computed once for all chunks.  Four channels per slot cut the
    // per-value index work and the slot registers by four.
    {
      constexpr int VS = 4;
      constexpr int NSL = kStageSlots / VS;
      const int gper = half_ps / VS;  // channel groups per staged point (padding included)
      const int nst = npts_halo * gper;
      int64_t goff[NSL];
      int loff[NSL], csl[NSL];
#pragma unroll
      for (int i = 0; i < NSL; ++i) {
        const int e = tid + 256 * i;
        goff[i] = -2;
        loff[i] = 0;
        csl[i] = 0;
        if (e < nst) {
          const int cs = (e % gper) * VS;
          const int pt = e / gper;
          const int hh2 = pt % a.h[2];
          const int q = pt / a.h[2];
          const int hh1 = q % a.h[1];
          const int hh0 = q / a.h[1];
          const int64_t i0 = wrap_index(a.org[0] + base0 + hh0, a.wp[0]);
          const int64_t i1 = wrap_index(a.org[1] + base1 + hh1, a.wp[1]);
          const int64_t i2 = wrap_index(a.org[2] + base2 + hh2, a.wp[2]);
          const bool ok = i0 >= a.vlo[0] && i0 < a.vhi[0] && i1 >= a.vlo[1] && i1 < a.vhi[1] && i2 >= a.vlo[2] &&
                          i2 < a.vhi[2];
          goff[i] = ok ? i0 * a.is[0] + i1 * a.is[1] + i2 * a.is[2] : -1;
          loff[i] = (hh0 * a.h[1] + hh1) * a.rs + hh2 * a.ps + 2 * cs;
          csl[i] = cs;
        }
      }
      float buf[NSL][2 * VS];
      auto load = [&](const int chg) {
        const int cbase = chg * a.chunk_c;
#pragma unroll
        for (int i = 0; i < NSL; ++i) {
          const int nv = (goff[i] >= 0 && csl[i] < a.chunk_c) ? max(0, min(VS, a.cin - (cbase + csl[i]))) : 0;
          load_unit<VS>(a.in, nv ? goff[i] + (cbase - a.chan_base) + csl[i] : 0, nv, buf[i]);
        }
      };
      auto store = [&]() {
#pragma unroll
        for (int i = 0; i < NSL; ++i)
          if (goff[i] != -2) stage_store<PREC, VS>(lds, lds_lo, loff[i], buf[i], in_sc);
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
  }

  // Epilogue: lane holds rows 4g..4g+3 (positions along axis 1) of column m
  // of each of its FM x FN tiles.  Launch column lc = delta * coutr + c.
  // Column terms are formed once per column, position terms once per
  // fragment; the four rows of a fragment step by one position along axis 1.
  // A k-split's waves add their tiles in wave order; wave ks finishes
  // fragments [ks FE, ks FE + FE) of its group.  Each wave passes the other
  // owners' blocks through LDS (slot o - (o > w) of writer w for owner o)
  // and keeps its own block in registers.
  float4_t eacc[FE][FN];
  if constexpr (KS == 1) {
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
      for (int j = 0; j < FN; ++j) eacc[f][j] = acc[f][j];
  } else {
    __syncthreads();  // every wave is done with the staged halo
    float* red = reinterpret_cast<float*>(smem);
    auto slot = [&](const int w, const int pos, const int fe, const int j, const int r) {
      return ((((((wgrp * KS + w) * (KS - 1) + pos) * FE + fe) * FN + j) * 4 + r) * 64) + lane;
    };
#pragma unroll
    for (int o = 0; o < KS; ++o) {
      if (o == ks) continue;  // wave-uniform
      const int pos = o - (o > ks ? 1 : 0);
#pragma unroll
      for (int fe = 0; fe < FE; ++fe)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) red[slot(ks, pos, fe, j, r)] = acc[o * FE + fe][j][r];
    }
    __syncthreads();
#pragma unroll
    for (int o = 0; o < KS; ++o) {
      if (o != ks) continue;  // wave-uniform: register indices stay static
#pragma unroll
      for (int fe = 0; fe < FE; ++fe)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float v = 0.f;
#pragma unroll
            for (int w = 0; w < KS; ++w) v += w == o ? acc[o * FE + fe][j][r] : red[slot(w, o - (o > w ? 1 : 0), fe, j, r)];
            eacc[fe][j][r] = v;
          }
    }
  }
  double ssq = 0.0;
  float vmax = 0.f;
  const int64_t r0 = base1 + 4 * g;  // axis-1 position of this lane's first row
  int cdel[FN];
  bool cok[FN];
  int64_t coff[FN];  // column offset in output elements (floats; halfwords for the compact residual)
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int lc = by * BC + (wc * FN + j) * 16 + m;
    cok[j] = lc < D * a.coutr;
    cdel[j] = D == 1 ? 0 : lc / a.coutr;
    const int c = lc - cdel[j] * a.coutr;
    if constexpr (YB == 2) {
      const int f = c >> 1;
      coff[j] = 2 * ((int64_t)(f / a.ybw) * a.yblk + f % a.ybw) + (c & 1);
    } else {
      coff[j] = c;
    }
  }
#pragma unroll
  for (int f = 0; f < FE; ++f) {
    const int fg = wr * FM + ks * FE + f;
    const int64_t p0 = base0 + fg / T2, p2b = base2 + (int64_t)(fg % T2) * D;
    const int64_t obase = p0 * a.os[0] + r0 * a.os[1] + p2b * a.os[2];
    const int64_t mbase = (a.morg[0] + p0) * a.ms[0] + (a.morg[1] + r0) * a.ms[1] + (a.morg[2] + p2b) * a.ms[2];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      if (!cok[j]) continue;
      if (p0 >= a.oe[0] || p2b + cdel[j] >= a.oe[2]) continue;
      const int64_t ob = obase + cdel[j] * a.os[2], mb = mbase + cdel[j] * a.ms[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (r0 + i >= a.oe[1]) continue;
        const bool masked = a.mask && a.mask[mb + i * a.ms[1]] != 0;
        float v = masked ? 0.f : eacc[f][j][i] * out_sc;
        if (a.out) {
          const int64_t q = ob + i * a.os[1];
          if constexpr (YB == 2) {
            reinterpret_cast<uint16_t*>(a.out)[2 * q + coff[j]] = (uint16_t)pack_bf16(v, 0.f);
          } else {
            float* dst = a.out + 2 * q + coff[j];
            if (a.accumulate) v += *dst;
            *dst = v;
          }
        }
        ssq += (double)v * (double)v;
        vmax = fmaxf(vmax, fabsf(v));
      }
    }
  }
  if (a.partial) {
    __shared__ double red[4];
    const double tot = block_sum_d(ssq, red);
    if (tid == 0) a.partial[(size_t)by * gx + bx] = tot;
  }
  if (a.absmax) {
    __shared__ float redm[4];
    for (int off = 32; off > 0; off >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, off, 64));
    if (lane == 0) redm[wave] = vmax;
    __syncthreads();
    if (tid == 0) a.absmax[(size_t)by * gx + bx] = fmaxf(fmaxf(redm[0], redm[1]), fmaxf(redm[2], redm[3]));
  }
}

// Workgroups are dispatched to the 8 XCDs round-robin; remap the linear id so
// that each XCD (own L2) processes a contiguous range of work items, whose
// neighbours then share staged input and weights through the same L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t w, int64_t W) {
  const int64_t per = W / 8, rem = W % 8;
  const int64_t xcd = w % 8, idx = w / 8;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// Work item lin -> (position tile, column block).  Tiles go in runs of
// `run`; inside a run the column blocks are the outer index, so one column
// block's weights stay in L2 while the run's tiles (whose staged input is
// also L2-resident) pass through it.  run = 1 is tile-major order.
__device__ __forceinline__ void split_work(const int64_t lin, const int64_t gx, const int gy, const int run,
                                           int64_t& tile, int& cb) {
  const int64_t per = (int64_t)run * gy;
  const int64_t first = lin / per * run;
  const int64_t width = min((int64_t)run, gx - first);
  const int64_t r = lin - first * gy;
  cb = (int)(r / width);
  tile = first + (r - (int64_t)cb * width);
}

template <int PREC, int T0, int T2, int WC, int FN, int D, int KS, bool PIPE, int YB = 0>
__global__ __launch_bounds__(256) void conv_kernel(ConvArgs a, int64_t gx, int gy, int run) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t lin = xcd_remap(blockIdx.x, gx * gy);
  int64_t tile;
  int cb;
  split_work(lin, gx, gy, run, tile, cb);
  conv_tile<PREC, T0, T2, WC, FN, D, KS, PIPE, YB>(a, tile, cb, gx, smem);
}

// Persistent batched launch: the work list is every (position tile, column
// block) of every problem; tile_start[q] is the first work item of problem
// q.  Workgroups stride over the list, so problems of any size and channel
// count share one launch.  Each item runs the same tile code as the
// per-problem kernel, so results are bitwise identical.
template <int PREC, int T0, int T2, int WC, int FN, int D, int KS, bool PIPE>
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
    conv_tile<PREC, T0, T2, WC, FN, D, KS, PIPE>(a, local % gx, (int)(local / gx), gx, smem);
    __syncthreads();  // the next item reuses LDS
  }
}

// Per-problem launches: one 1-D grid of gx * gy workgroups.
template <int PREC>
int32_t launch_prec_impl(const ConvPlan& p, bool pipe, hipStream_t st) {
  const dim3 grid((unsigned)(p.gx * p.gy)), block(256);
  switch (p.tile) {
#define HICU_TILE_CASE(id, T0, T2, WC, FN, D, KS, P, B)                                                            \
  case id:                                                                                                     \
    if constexpr (PREC == P_BF16 && T0 > 1) {                                                                  \
      if (p.a.yb == 1) {                                                                                       \
        hipLaunchKernelGGL((conv_kernel<PREC, T0, T2, WC, FN, D, KS, false, 1>), grid, block, p.lds_bytes, st, p.a, \
                           p.gx, p.gy, p.run);                                                                 \
        break;                                                                                                 \
      }                                                                                                        \
      if (p.a.yb == 2) {                                                                                       \
        hipLaunchKernelGGL((conv_kernel<PREC, T0, T2, WC, FN, D, KS, false, 2>), grid, block, p.lds_bytes, st, p.a, \
                           p.gx, p.gy, p.run);                                                                 \
        break;                                                                                                 \
      }                                                                                                        \
    }                                                                                                          \
    if (p.a.yb != 0) return HICU_ERR_UNSUPPORTED;                                                              \
    if constexpr (P != 0) {                                                                                    \
      if (pipe) {                                                                                              \
        hipLaunchKernelGGL((conv_kernel<PREC, T0, T2, WC, FN, D, KS, true>), grid, block, p.lds_bytes, st, p.a,     \
                           p.gx, p.gy, p.run);                                                                 \
        break;                                                                                                 \
      }                                                                                                        \
    }                                                                                                          \
    hipLaunchKernelGGL((conv_kernel<PREC, T0, T2, WC, FN, D, KS, false>), grid, block, p.lds_bytes, st, p.a, p.gx,  \
                       p.gy, p.run);                                                                           \
    break;
    HICU_TILES(HICU_TILE_CASE)
#undef HICU_TILE_CASE
    default:
      return HICU_ERR_UNSUPPORTED;
  }
  return HICU_OK;
}

template <int PREC>
int32_t launch_batch_prec_impl(const BatchConvLaunch& b, hipStream_t st) {
  const dim3 grid(b.grid), block(256);
  switch (b.tile) {
#define HICU_TILE_CASE(id, T0, T2, WC, FN, D, KS, P, B)                                                          \
  case id:                                                                                                   \
    if constexpr (B != 0) {                                                                                  \
      if (b.pipe)                                                                                            \
        hipLaunchKernelGGL((conv_batch_kernel<PREC, T0, T2, WC, FN, D, KS, true>), grid, block, b.lds_bytes, st,  \
                           b.args, b.tile_start, b.nprob, b.total);                                          \
      else                                                                                                   \
        hipLaunchKernelGGL((conv_batch_kernel<PREC, T0, T2, WC, FN, D, KS, false>), grid, block, b.lds_bytes, st, \
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

}  // namespace hicu
