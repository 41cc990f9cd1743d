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

template <int PREC>
__device__ __forceinline__ void stage_store(typename LdsElem<PREC>::T* hi, typename LdsElem<PREC>::T* lo,
                                            int64_t off, float2 v) {
  if constexpr (PREC == P_F32) {
    *reinterpret_cast<float2*>(hi + off) = v;
  } else if constexpr (PREC == P_BF16) {
    const uint32_t w = (uint32_t)f2bf(v.x) | ((uint32_t)f2bf(v.y) << 16);
    *reinterpret_cast<uint32_t*>(hi + off) = w;
  } else {
    const uint16_t hx = f2bf(v.x), hy = f2bf(v.y);
    const uint16_t lx = f2bf(v.x - bf2f(hx)), ly = f2bf(v.y - bf2f(hy));
    *reinterpret_cast<uint32_t*>(hi + off) = (uint32_t)hx | ((uint32_t)hy << 16);
    *reinterpret_cast<uint32_t*>(lo + off) = (uint32_t)lx | ((uint32_t)ly << 16);
  }
}

// PIPE: stage channel chunks through registers, prefetching chunk c + 1 from
// global memory while chunk c is multiplied (used when several chunks are
// streamed and a chunk fits in kStageSlots complex values per thread).
constexpr int kStageSlots = 16;

// One output tile: positions tile bx (of gx along the position grid) and
// column block by.  Shared by the per-problem kernel and the persistent
// batched kernel.
template <int PREC, int T0, int T2, int WN, bool PIPE>
__device__ __forceinline__ void conv_tile(const ConvArgs& a, const int64_t bx, const int by, const int64_t gx,
                                          unsigned char* smem) {
  constexpr int KB = kblock_of(PREC);
  constexpr int NFRAG = T0 * T2;
  static_assert(NFRAG % 4 == 0, "tile must give each wave whole fragments");
  constexpr int WM = NFRAG / 4;
  constexpr bool SPLIT = PREC == P_BF16X3;
  using E = typename LdsElem<PREC>::T;

  E* lds = reinterpret_cast<E*>(smem);
  const int64_t lds_elems = (int64_t)a.h[0] * a.h[1] * a.rs;
  E* lds_lo = lds + lds_elems;

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, m = lane & 15;
  const int64_t t2i = bx % a.nt[2];
  const int64_t t1i = (bx / a.nt[2]) % a.nt[1];
  const int64_t t0i = bx / (a.nt[2] * a.nt[1]);
  const int64_t base0 = t0i * T0, base1 = t1i * 16, base2 = t2i * T2;
  const int n0 = a.col0 + by * (16 * WN);

  // Row tails (read with zero weights) must hold finite values.
  {
    const int tail = a.rs - a.h[2] * a.ps;
    const int nrows = a.h[0] * a.h[1];
    for (int e = tid; e < nrows * tail; e += 256) {
      const int64_t off = (int64_t)(e / tail) * a.rs + a.h[2] * a.ps + (e % tail);
      lds[off] = E(0);
      if constexpr (SPLIT) lds_lo[off] = E(0);
    }
  }

  float4_t acc[WM][WN];
#pragma unroll
  for (int f = 0; f < WM; ++f)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[f][j] = float4_t{0.f, 0.f, 0.f, 0.f};

  // Per-fragment LDS offsets of this lane's operand (without kernel shift).
  int frag_off[WM];
#pragma unroll
  for (int f = 0; f < WM; ++f) {
    const int fg = wave * WM + f;
    const int fa = fg / T2, fc = fg % T2;
    frag_off[f] = (fa * a.h[1] + m) * a.rs + fc * a.ps + g * (KB / 4);
  }

  const int half_ps = a.ps >> 1;
  const int64_t npts_halo = (int64_t)a.h[0] * a.h[1] * a.h[2];
  const int64_t nstage = npts_halo * half_ps;

  auto compute_chunk = [&](const int chg) {
    for (int k0 = 0; k0 < a.k[0]; ++k0) {
      for (int k1 = 0; k1 < a.k[1]; ++k1) {
        const int shift = (k0 * a.h[1] + k1) * a.rs;
        const size_t wrow = ((((size_t)chg * a.k[0] + k0) * a.k[1] + k1) * a.nkb) * a.ncolp;
        for (int t = 0; t < a.nkb; ++t) {
          const size_t wt = (wrow + (size_t)t * a.ncolp + n0 + m) * KB + g * (KB / 4);
          if constexpr (PREC == P_F32) {
            float4_t av[WM], bv[WN];
#pragma unroll
            for (int f = 0; f < WM; ++f)
              av[f] = *reinterpret_cast<const float4_t*>(lds + frag_off[f] + shift + t * KB);
            const float* Bp = reinterpret_cast<const float*>(a.B);
#pragma unroll
            for (int j = 0; j < WN; ++j)
              bv[j] = *reinterpret_cast<const float4_t*>(Bp + wt + (size_t)j * 16 * KB);
#pragma unroll
            for (int f = 0; f < WM; ++f)
#pragma unroll
              for (int j = 0; j < WN; ++j) {
                acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[f][0], bv[j][0], acc[f][j], 0, 0, 0);
                acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[f][1], bv[j][1], acc[f][j], 0, 0, 0);
                acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[f][2], bv[j][2], acc[f][j], 0, 0, 0);
                acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[f][3], bv[j][3], acc[f][j], 0, 0, 0);
              }
          } else {
            bf16x8_t av[WM], bv[WN];
#pragma unroll
            for (int f = 0; f < WM; ++f)
              av[f] = __builtin_bit_cast(
                  bf16x8_t, *reinterpret_cast<const u32x4_t*>(lds + frag_off[f] + shift + t * KB));
            const uint16_t* Bp = reinterpret_cast<const uint16_t*>(a.B);
#pragma unroll
            for (int j = 0; j < WN; ++j)
              bv[j] = __builtin_bit_cast(bf16x8_t,
                                         *reinterpret_cast<const u32x4_t*>(Bp + wt + (size_t)j * 16 * KB));
#pragma unroll
            for (int f = 0; f < WM; ++f)
#pragma unroll
              for (int j = 0; j < WN; ++j)
                acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[f], bv[j], acc[f][j], 0, 0, 0);
            if constexpr (SPLIT) {
              bf16x8_t al[WM], bl[WN];
#pragma unroll
              for (int f = 0; f < WM; ++f)
                al[f] = __builtin_bit_cast(
                    bf16x8_t, *reinterpret_cast<const u32x4_t*>(lds_lo + frag_off[f] + shift + t * KB));
              const uint16_t* Bl = reinterpret_cast<const uint16_t*>(a.Blo);
#pragma unroll
              for (int j = 0; j < WN; ++j)
                bl[j] = __builtin_bit_cast(
                    bf16x8_t, *reinterpret_cast<const u32x4_t*>(Bl + wt + (size_t)j * 16 * KB));
#pragma unroll
              for (int f = 0; f < WM; ++f)
#pragma unroll
                for (int j = 0; j < WN; ++j) {
                  acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[f], bl[j], acc[f][j], 0, 0, 0);
                  acc[f][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[f], bv[j], acc[f][j], 0, 0, 0);
                }
            }
          }
        }
      }
    }
  };

  if constexpr (!PIPE) {
    for (int ch = 0; ch < a.nchunks; ++ch) {
      const int chg = a.ch0 + ch;
      const int cbase = chg * a.chunk_c;
      __syncthreads();
      for (int64_t e = tid; e < nstage; e += 256) {
        const int cs = (int)(e % half_ps);
        const int64_t pt = e / half_ps;
        const int hh2 = (int)(pt % a.h[2]);
        const int64_t q = pt / a.h[2];
        const int hh1 = (int)(q % a.h[1]);
        const int hh0 = (int)(q / a.h[1]);
        const int64_t i0 = a.org[0] + base0 + hh0;
        const int64_t i1 = a.org[1] + base1 + hh1;
        const int64_t i2 = a.org[2] + base2 + hh2;
        const int ci = cbase + cs;
        float2 v = make_float2(0.f, 0.f);
        if (cs < a.chunk_c && ci < a.cin && i0 >= a.vlo[0] && i0 < a.vhi[0] && i1 >= a.vlo[1] &&
            i1 < a.vhi[1] && i2 >= a.vlo[2] && i2 < a.vhi[2])
          v = a.in[i0 * a.is[0] + i1 * a.is[1] + i2 * a.is[2] + (ci - a.chan_base)];
        const int64_t off = ((int64_t)hh0 * a.h[1] + hh1) * a.rs + (int64_t)hh2 * a.ps + 2 * cs;
        stage_store<PREC>(lds, lds_lo, off, v);
      }
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
      const int64_t e = tid + 256 * i;
      goff[i] = -2;
      loff[i] = 0;
      csl[i] = 0;
      if (e < nstage) {
        const int cs = (int)(e % half_ps);
        const int64_t pt = e / half_ps;
        const int hh2 = (int)(pt % a.h[2]);
        const int64_t q = pt / a.h[2];
        const int hh1 = (int)(q % a.h[1]);
        const int hh0 = (int)(q / a.h[1]);
        const int64_t i0 = a.org[0] + base0 + hh0;
        const int64_t i1 = a.org[1] + base1 + hh1;
        const int64_t i2 = a.org[2] + base2 + hh2;
        const bool ok = i0 >= a.vlo[0] && i0 < a.vhi[0] && i1 >= a.vlo[1] && i1 < a.vhi[1] && i2 >= a.vlo[2] &&
                        i2 < a.vhi[2];
        goff[i] = ok ? i0 * a.is[0] + i1 * a.is[1] + i2 * a.is[2] : -1;
        loff[i] = (int)(((int64_t)hh0 * a.h[1] + hh1) * a.rs + (int64_t)hh2 * a.ps + 2 * cs);
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
        if (goff[i] != -2) stage_store<PREC>(lds, lds_lo, loff[i], buf[i]);
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

  // Epilogue: lane holds rows 4g..4g+3 (positions along axis 1) of column m.
  double ssq = 0.0;
#pragma unroll
  for (int f = 0; f < WM; ++f) {
    const int fg = wave * WM + f;
    const int64_t p0 = base0 + fg / T2, p2 = base2 + fg % T2;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t p1 = base1 + 4 * g + i;
      const bool pv = p0 < a.oe[0] && p1 < a.oe[1] && p2 < a.oe[2];
      if (!pv) continue;
      bool masked = false;
      if (a.mask)
        masked = a.mask[(a.morg[0] + p0) * a.ms[0] + (a.morg[1] + p1) * a.ms[1] + (a.morg[2] + p2) * a.ms[2]] != 0;
      const int64_t ob = 2 * (p0 * a.os[0] + p1 * a.os[1] + p2 * a.os[2]);
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        const int lc = by * (16 * WN) + j * 16 + m;
        if (lc >= a.coutr) continue;
        float v = masked ? 0.f : acc[f][j][i] * a.scale;
        if (a.out) {
          float* dst = a.out + ob + lc;
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

template <int PREC, int T0, int T2, int WN, bool PIPE>
__global__ __launch_bounds__(256) void conv_kernel(ConvArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  conv_tile<PREC, T0, T2, WN, PIPE>(a, blockIdx.x, blockIdx.y, gridDim.x, smem);
}

// Persistent batched launch: the work list is every (position tile, column
// block) of every problem; tile_start[q] is the first work item of problem
// q.  Workgroups stride over the list, so problems of any size and channel
// count share one launch.  Each item runs the same tile code as the
// per-problem kernel, so results are bitwise identical.
template <int PREC, int T0, int T2, int WN, bool PIPE>
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
    conv_tile<PREC, T0, T2, WN, PIPE>(a, local % gx, (int)(local / gx), gx, smem);
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
  const int kk2 = run / a.ps, el = run % a.ps;
  float v = 0.f;
  if (kk2 < a.k2 && el < 2 * a.chunk_c && col < a.coutr_total) {
    const int ci = ch * a.chunk_c + (el >> 1), ri = el & 1;
    const int co = col >> 1, ro = col & 1;
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
WeightShape weight_shape(int prec, const int k[3], int cin, int chunk_c, int coutr_total) {
  WeightShape w;
  w.KB = kblock_of(prec);
  w.chunk_c = chunk_c;
  w.nchunks = (int)cdiv(cin, chunk_c);
  w.ps = (int)rup(2 * chunk_c, 8);
  w.nkb = (int)cdiv((int64_t)k[2] * w.ps, w.KB);
  w.ncolp = (int)rup(coutr_total, kColPad);
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
  a.total = (int64_t)ws.elems;
  a.B = B;
  a.Blo = Blo;
  return a;
}

int32_t launch_prep_weights(int mode, int prec, const Geo& g, const float2* F, int p,
                            const WeightShape& ws, void* B, void* Blo, hipStream_t st) {
  const PrepArgs a = make_prep_args(mode, prec, g, F, p, ws, B, Blo);
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

template <int PREC, int T0, int T2, int WN, bool PIPE>
static void launch_batch_inst(const BatchConvLaunch& b, hipStream_t st) {
  hipLaunchKernelGGL((conv_batch_kernel<PREC, T0, T2, WN, PIPE>), dim3(b.grid), dim3(256), b.lds_bytes, st, b.args,
                     b.tile_start, b.nprob, b.total);
}

template <int PREC, int T0, int T2, bool PIPE>
static void launch_batch_wn(const BatchConvLaunch& b, hipStream_t st) {
  switch (b.t.WN) {
    case 1: launch_batch_inst<PREC, T0, T2, 1, PIPE>(b, st); break;
    case 2: launch_batch_inst<PREC, T0, T2, 2, PIPE>(b, st); break;
    default: launch_batch_inst<PREC, T0, T2, 4, PIPE>(b, st); break;
  }
}

template <int PREC, int T0, int T2>
static void launch_batch_pipe(const BatchConvLaunch& b, hipStream_t st) {
  if (b.pipe) launch_batch_wn<PREC, T0, T2, true>(b, st);
  else launch_batch_wn<PREC, T0, T2, false>(b, st);
}

template <int PREC>
static int32_t launch_batch_prec(const BatchConvLaunch& b, hipStream_t st) {
  const int T0 = b.t.T0, T2 = b.t.T2;
  if (T0 == 1 && T2 == 4) launch_batch_pipe<PREC, 1, 4>(b, st);
  else if (T0 == 1 && T2 == 8) launch_batch_pipe<PREC, 1, 8>(b, st);
  else if (T0 == 2 && T2 == 4) launch_batch_pipe<PREC, 2, 4>(b, st);
  else if (T0 == 2 && T2 == 8) launch_batch_pipe<PREC, 2, 8>(b, st);
  else return HICU_ERR_UNSUPPORTED;
  return HICU_OK;
}

int32_t launch_conv_batch(const BatchConvLaunch& b, hipStream_t st) {
  if (b.nprob < 1 || b.total < 1 || b.grid < 1) return HICU_ERR_ARG;
  int32_t s;
  if (b.prec == P_F32) s = launch_batch_prec<P_F32>(b, st);
  else if (b.prec == P_BF16) s = launch_batch_prec<P_BF16>(b, st);
  else s = launch_batch_prec<P_BF16X3>(b, st);
  if (s != HICU_OK) return s;
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

bool conv_can_pipe(const ConvPlan& p) {
  const int64_t nstage = (int64_t)p.a.h[0] * p.a.h[1] * p.a.h[2] * (p.a.ps / 2);
  return nstage <= 256 * kStageSlots;
}

TileCfg default_tile(int prec, const Geo& g, int coutr) {
  (void)prec;
  const int WN = coutr <= 16 ? 1 : (coutr <= 32 ? 2 : 4);
  if (g.k[0] == 1) return TileCfg{1, 8, WN};
  return TileCfg{2, 4, WN};
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

int32_t plan_conv(int prec, TileCfg t, const int k[3], const WeightShape& ws, int nchunks,
                  const int64_t oe[3], int coutr, ConvPlan* plan) {
  if (t.T0 < 1 || t.T2 < 1 || (t.T0 * t.T2) % 4 != 0 || t.WN < 1 || t.WN > 4) return HICU_ERR_ARG;
  ConvArgs& a = plan->a;
  plan->prec = prec;
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
  a.h[2] = t.T2 + k[2] - 1;
  const int need = (t.T2 - 1) * ws.ps + ws.nkb * ws.KB;
  a.rs = pick_rs(prec, need);
  const size_t esize = prec == P_F32 ? 4 : 2;
  plan->lds_bytes = (size_t)a.h[0] * a.h[1] * a.rs * esize * (prec == P_BF16X3 ? 2 : 1);
  if (plan->lds_bytes > 65536) return HICU_ERR_UNSUPPORTED;
  a.oe[0] = oe[0];
  a.oe[1] = oe[1];
  a.oe[2] = oe[2];
  a.nt[0] = cdiv(oe[0], t.T0);
  a.nt[1] = cdiv(oe[1], 16);
  a.nt[2] = cdiv(oe[2], t.T2);
  const int64_t gx = a.nt[0] * a.nt[1] * a.nt[2];
  const int64_t gy = cdiv(coutr, 16 * t.WN);
  if (gx <= 0 || gx > 0x7fffffff || gy <= 0 || gy > 65535) return HICU_ERR_SHAPE;
  a.coutr = coutr;
  plan->grid = dim3((unsigned)gx, (unsigned)gy, 1);
  return HICU_OK;
}

template <int PREC, int T0, int T2, bool PIPE>
static void launch_wn(const ConvPlan& p, hipStream_t st) {
  switch (p.t.WN) {
    case 1: hipLaunchKernelGGL((conv_kernel<PREC, T0, T2, 1, PIPE>), p.grid, dim3(256), p.lds_bytes, st, p.a); break;
    case 2: hipLaunchKernelGGL((conv_kernel<PREC, T0, T2, 2, PIPE>), p.grid, dim3(256), p.lds_bytes, st, p.a); break;
    default: hipLaunchKernelGGL((conv_kernel<PREC, T0, T2, 4, PIPE>), p.grid, dim3(256), p.lds_bytes, st, p.a); break;
  }
}

template <int PREC, int T0, int T2>
static void launch_pipe(const ConvPlan& p, hipStream_t st) {
  const int64_t nstage = (int64_t)p.a.h[0] * p.a.h[1] * p.a.h[2] * (p.a.ps / 2);
  if (p.a.nchunks > 1 && nstage <= 256 * kStageSlots) launch_wn<PREC, T0, T2, true>(p, st);
  else launch_wn<PREC, T0, T2, false>(p, st);
}

template <int PREC>
static int32_t launch_prec(const ConvPlan& p, hipStream_t st) {
  const int T0 = p.t.T0, T2 = p.t.T2;
  if (T0 == 1 && T2 == 4) launch_pipe<PREC, 1, 4>(p, st);
  else if (T0 == 1 && T2 == 8) launch_pipe<PREC, 1, 8>(p, st);
  else if (T0 == 2 && T2 == 4) launch_pipe<PREC, 2, 4>(p, st);
  else if (T0 == 2 && T2 == 8) launch_pipe<PREC, 2, 8>(p, st);
  else return HICU_ERR_UNSUPPORTED;
  return HICU_OK;
}

int32_t launch_conv(const ConvPlan& p, hipStream_t st) {
  // Host-side guard of every index the kernel forms from its arguments.
  const ConvArgs& a = p.a;
  if ((int64_t)a.col0 + (int64_t)p.grid.y * 16 * p.t.WN > a.ncolp) return HICU_ERR_SHAPE;
  if (a.ps < 2 * a.chunk_c || a.ps % 8 != 0) return HICU_ERR_SHAPE;
  if (a.rs < (p.t.T2 - 1) * a.ps + a.nkb * kblock_of(p.prec)) return HICU_ERR_SHAPE;
  if (a.nkb * kblock_of(p.prec) < a.k[2] * a.ps) return HICU_ERR_SHAPE;
  if ((int64_t)a.ch0 * a.chunk_c < a.chan_base) return HICU_ERR_SHAPE;
  int32_t s;
  if (p.prec == P_F32) s = launch_prec<P_F32>(p, st);
  else if (p.prec == P_BF16) s = launch_prec<P_BF16>(p, st);
  else s = launch_prec<P_BF16X3>(p, st);
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
