// Host side of the contraction kernels (planning, weight builder, launch
// dispatch); the kernels themselves are in conv_impl.h, instantiated per
// precision in conv_f32.hip, conv_bf16.hip, conv_bf16x3.hip and conv_f16.hip.
#include <algorithm>

#include "conv.h"

namespace hicu {

template <int PREC> int32_t launch_prec_impl(const ConvPlan& p, bool pipe, hipStream_t st);
template <int PREC> int32_t launch_batch_prec_impl(const BatchConvLaunch& b, hipStream_t st);
extern template int32_t launch_prec_impl<P_F32>(const ConvPlan&, bool, hipStream_t);
extern template int32_t launch_prec_impl<P_BF16>(const ConvPlan&, bool, hipStream_t);
extern template int32_t launch_prec_impl<P_BF16X3>(const ConvPlan&, bool, hipStream_t);
extern template int32_t launch_prec_impl<P_F16>(const ConvPlan&, bool, hipStream_t);
extern template int32_t launch_batch_prec_impl<P_F32>(const BatchConvLaunch&, hipStream_t);
extern template int32_t launch_batch_prec_impl<P_BF16>(const BatchConvLaunch&, hipStream_t);
extern template int32_t launch_batch_prec_impl<P_BF16X3>(const BatchConvLaunch&, hipStream_t);

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
  } else if (a.prec == P_F16) {
    reinterpret_cast<_Float16*>(a.B)[e] = (_Float16)v;
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
#define HICU_TILE_ROW(id, T0, T2, WC, FN, D, KS, P, B) {T0, T2, WC, FN, D, KS},
      HICU_TILES(HICU_TILE_ROW)
#undef HICU_TILE_ROW
  };
  return (id >= 0 && id < kNumTiles) ? table[id] : TileCfg{0, 0, 0, 0, 0, 1};
}

bool tile_batch_ok(int id) {
  static const bool table[kNumTiles] = {
#define HICU_TILE_ROW(id, T0, T2, WC, FN, D, KS, P, B) B != 0,
      HICU_TILES(HICU_TILE_ROW)
#undef HICU_TILE_ROW
  };
  return id >= 0 && id < kNumTiles && table[id];
}

static bool tile_pipe_ok(int id) {
  static const bool table[kNumTiles] = {
#define HICU_TILE_ROW(id, T0, T2, WC, FN, D, KS, P, B) P != 0,
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

bool compact_tile_ok(const ConvPlan& p) {
  const TileCfg t = tile_cfg(p.tile);
  return p.prec == P_BF16 && t.T0 > 1;
}

int conv_vec(const ConvArgs& a) {
  const bool aligned = (reinterpret_cast<uintptr_t>(a.in) & 15) == 0;
  for (int V : {4, 2}) {
    if (aligned && a.is[2] % V == 0 && a.chunk_c % V == 0 && a.chan_base % V == 0) return V;
  }
  return 1;
}

int32_t launch_conv_batch(const BatchConvLaunch& b, hipStream_t st) {
  if (b.nprob < 1 || b.total < 1 || b.grid < 1) return HICU_ERR_ARG;
  if (b.lds_bytes > kMaxLds) return HICU_ERR_UNSUPPORTED;
  int32_t s;
  if (b.prec == P_F16) return HICU_ERR_UNSUPPORTED;
  if (b.prec == P_F32) s = launch_batch_prec_impl<P_F32>(b, st);
  else if (b.prec == P_BF16) s = launch_batch_prec_impl<P_BF16>(b, st);
  else s = launch_batch_prec_impl<P_BF16X3>(b, st);
  if (s != HICU_OK) return s;
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

// Shapes tried first, from timings of every shape on the 256 x 232 x 16-coil
// 2-D workload and a 64 x 80 x 80 x 8-coil volume with a 5 x 5 x 5 kernel:
// the forward (many columns) takes the 2 x 2 wave grid, the narrow adjoint
// one or two column fragments per wave without axis-2 packing (the packed
// shapes lengthen the reduction by (k2 + D - 1) / k2 and were slower once
// operand fetch stopped being the limit).  The BF16 volume adjoint, which
// reads the compact BF16 residual with batched staging loads, takes
// 8 planes x 16 x 2 pairs packed along axis 2 (D = 2: with 8-channel chunks
// the widened 6-tap run fills the same three k-blocks as 5 taps), timed on
// a 64 x 320 x 320 x 8 slab with 900 filters at 62.1 ms, against 66.4 ms for
// 8 x 16 x 4 unpacked and 76.2 ms for 2 x 16 x 8.  Its forward, which writes
// that residual, takes 4 x 16 x 4 positions by 64 columns on a 2 x 2 wave
// grid (8 x 2 fragments per wave: half the weight loads per MFMA of the
// 4 x 4 register tiles), 49.3 ms against 53.9 ms for 2 x 16 x 8 with one
// wave column and 57.8 ms for 2 x 16 x 4 by 128; the line search over all
// filters, which shares the shape, 43.5 against 47.9 ms.
// The planar adjoint with two column fragments (32 real outputs) splits
// the k-steps over the waves: on the 16-coil workload with 280 filters
// the BF16 adjoint takes 97 us with 8 fragments per wave and KS = 4,
// against 153 us for 2 fragments per wave; FP32 502 against 530 us; the
// split BF16 pair, whose two operand sets make 8 x 2 fragments too many,
// 166 us with KS = 2 against 232 us.  Volume adjoints keep their shapes:
// there every k-split shape timed slower (48 ms and up on the 64-plane
// slab against 32.4 ms).
int default_tile(int prec, const Geo& g, int coutr, int role) {
  const bool is3d = g.k[0] > 1;
  const int frags = (int)cdiv(coutr, 16);
  if (role == 1) {
    if (is3d) return frags >= 3 ? 15 : (frags == 2 ? 14 : (prec == P_F32 ? 13 : (prec == P_BF16 ? 31 : 16)));
    if (frags == 2) return prec == P_BF16X3 ? 42 : (prec == P_F16 ? 1 : 36);
    return frags >= 3 ? 2 : 0;
  }
  if (frags >= 8) return is3d ? (prec == P_BF16 ? 35 : 19) : (prec == P_F32 ? 6 : (prec == P_BF16X3 ? 2 : 7));
  if (frags >= 3) return is3d ? 15 : 2;
  if (frags == 2) return is3d ? 14 : 1;
  return is3d ? 13 : 0;
}

// LDS row stride: a 16-lane row of MFMA operand reads (16 bytes each, one
// per halo row) is conflict-free when the stride is an odd multiple of 16
// bytes: 4 mod 8 floats, 8 mod 16 halfwords.
static int pick_rs(int prec, int need) {
  if (prec == P_F32) {
    int rs = (int)rup(need, 4);
    while (rs % 8 != 4) rs += 4;
    return rs;
  }
  int rs = (int)rup(need, 8);
  while (rs % 16 != 8) rs += 8;
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
  a.yb = 0;
  a.ybw = 0;
  a.yblk = 0;
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
  // wave k-split: the waves' partial tiles meet in LDS (after the last chunk)
  if (t.KS > 1) plan->lds_bytes = std::max(plan->lds_bytes, ks_reduce_bytes(t));
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
  // Weights that do not fit comfortably in one XCD's 4 MB L2 next to the
  // staged inputs are walked one column block at a time over runs of tiles.
  const size_t wbytes = (size_t)ws.elems * (prec == P_F32 ? 4 : 2) * (prec == P_BF16X3 ? 2 : 1);
  plan->run = 1;
  if (gy > 1 && wbytes > kL2Resident) plan->run = (int)std::min<int64_t>(gx, kTileRun);
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
  if (a.yb != 0) {
    if (!compact_tile_ok(p) || a.ybw < 1 || a.yblk < 0) return HICU_ERR_UNSUPPORTED;
    if (a.yb == 1 && (a.ybw != a.chunk_c || a.chan_base % a.chunk_c != 0)) return HICU_ERR_SHAPE;
    if (a.yb == 2 && a.accumulate) return HICU_ERR_UNSUPPORTED;
    if (a.yb != 1 && a.yb != 2) return HICU_ERR_ARG;
  }
  ConvPlan q = p;
  q.a.vec = conv_vec(a);
  // pipelined staging moves four aligned channels per slot
  const bool pipe = a.yb == 0 && a.nchunks > 1 && conv_can_pipe(p) && q.a.vec == 4;
  int32_t s;
  if (p.prec == P_F16) s = launch_prec_impl<P_F16>(q, pipe, st);
  else if (p.prec == P_F32) s = launch_prec_impl<P_F32>(q, pipe, st);
  else if (p.prec == P_BF16) s = launch_prec_impl<P_BF16>(q, pipe, st);
  else s = launch_prec_impl<P_BF16X3>(q, pipe, st);
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
