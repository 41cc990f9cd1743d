// Valid multi-channel correlation on MFMA: the im2col contraction behind the
// forward convolution H(x)F, the adjoint H'(Y F^H) and the line-search
// convolution H(g)F (THEORY section: HICU relies exclusively on these
// multi-dimensional convolutions).
#pragma once

#include "common.h"

namespace hicu {

// One launch computes, for every output position u in a box of extents oe
// and every real output column n in [col0, col0 + coutr):
//   out[u, n] = scale * sum_{k in kernel box} sum_{e} in[org + u + k, e] * W[k, e, n]
// where e runs over the real (re, im) entries of the input channels and
// input points outside the validity box [vlo, vhi) read as zero.  On an
// axis with period wp > 0 the input index org + u + k is first wrapped into
// [0, wp) (it lies within one period of that range).  Optional
// epilogue: zero at masked positions, add to the existing output, and a
// per-block sum of squares of the final values.
struct ConvArgs {
  const float2* in;
  int64_t is[3];          // input strides (complex elements) per spatial axis
  int cin;                // input channels are [chan_base, cin) (channel stride 1)
  int chan_base;          // channel index stored at offset 0 of each input point
  int vec;                // channels per staged unit (4, 2 or 1; see conv_vec)
  int chunk_c;            // complex channels per LDS chunk
  int nchunks;            // chunks processed by this launch
  int ch0;                // first input chunk (and weight chunk) of this launch
  int ps;                 // LDS elements per point (>= 2*chunk_c, multiple of 8)
  int nkb;                // k-blocks per contiguous run of k2*ps elements
  int rs;                 // LDS elements per halo row
  int h[3];               // halo extents
  int64_t vlo[3], vhi[3];
  int64_t org[3];
  int64_t wp[3] = {0, 0, 0};  // circular axis: input index taken modulo wp (then checked against vlo/vhi)
  int64_t oe[3];          // output extents
  int64_t nt[3];          // tiles per axis
  int k[3];
  const void* B;          // weights [chunk][k0][k1][kb][ncolp][KB]
  const void* Blo;        // low parts for the split precision
  int ncolp;              // padded weight columns
  int col0;               // first weight column of this launch
  int coutr;              // real output columns written by this launch
  float* out;             // real view of complex output, may be null
  int64_t os[3];          // output strides (complex elements)
  const uint8_t* mask;    // may be null
  int64_t ms[3];
  int64_t morg[3];        // mask coordinate of output position 0
  float scale;
  int accumulate;
  double* partial;        // per-block sum of squares, may be null
  const float* in_scale;  // FP16: device power of two applied to the staged input (undone in the epilogue)
  float* absmax;          // per-block max |output|, may be null
  // Compact residual (BF16 operands only): yb = 1 reads the input, yb = 2
  // writes the output as BF16 (re, im) pairs in blocks of ybw channels,
  // block b at complex offset b * yblk, points strided by is / os within a
  // block.  yb = 0: complex64, channels fastest.
  int yb;
  int ybw;
  int64_t yblk;
};

// Tile shapes.  A block of 4 waves owns T0 positions along axis 0, 16
// along axis 1 and T2*D along axis 2, and 16*WC*FN launch columns.  Its
// T0*T2 row fragments (16 positions each) are split over 4/(WC*KS) wave
// rows, its column fragments over WC wave columns, so each wave
// accumulates an FM x FN grid of 16 x 16 MFMA tiles (FM = T0*T2*WC*KS/4).
// KS > 1 splits the k-steps instead: the KS waves of a group take every
// KS-th k-step of each chunk for the same fragments, and their sums are
// added through LDS in wave order before the epilogue (narrow outputs
// then issue KS times more MFMAs per operand fetch and load each weight
// fragment once per block).  D > 1 packs D
// neighbouring outputs along axis 2 into the columns: launch column
// delta*coutr + c is output column c at axis-2 offset delta, computed with
// the kernel widened to k2 + D - 1 taps whose weights are shifted copies
// (zero outside the original taps).  Narrow outputs (the adjoint has only
// 2*coils real columns) then reuse every staged operand D times more.
struct TileCfg {
  int T0, T2, WC, FN, D, KS;
};

// X-macro list of the instantiated shapes: X(id, T0, T2, WC, FN, D, KS,
// pipelined staging available, batched kernel available).
#define HICU_TILES(X)            \
  X(0, 1, 8, 1, 1, 1, 1, 1, 1)   \
  X(1, 1, 8, 1, 2, 1, 1, 1, 1)   \
  X(2, 1, 8, 1, 4, 1, 1, 1, 1)   \
  X(3, 1, 4, 1, 1, 1, 1, 1, 1)   \
  X(4, 1, 4, 1, 2, 1, 1, 1, 1)   \
  X(5, 1, 4, 1, 4, 1, 1, 1, 1)   \
  X(6, 1, 8, 2, 2, 1, 1, 0, 0)   \
  X(7, 1, 8, 2, 4, 1, 1, 0, 0)   \
  X(8, 1, 16, 2, 4, 1, 1, 0, 0)   \
  X(9, 1, 16, 1, 2, 1, 1, 1, 1)   \
  X(10, 1, 8, 1, 4, 2, 1, 1, 0)   \
  X(11, 1, 16, 1, 4, 2, 1, 1, 0)   \
  X(12, 1, 8, 1, 4, 4, 1, 1, 0)   \
  X(13, 2, 4, 1, 1, 1, 1, 1, 1)   \
  X(14, 2, 4, 1, 2, 1, 1, 1, 1)   \
  X(15, 2, 4, 1, 4, 1, 1, 1, 1)   \
  X(16, 2, 8, 1, 1, 1, 1, 1, 0)   \
  X(17, 2, 8, 1, 2, 1, 1, 1, 0)   \
  X(18, 2, 8, 1, 4, 1, 1, 1, 0)   \
  X(19, 2, 4, 2, 4, 1, 1, 0, 0)   \
  X(20, 2, 8, 2, 4, 1, 1, 0, 0)   \
  X(21, 2, 4, 1, 4, 4, 1, 1, 0)   \
  X(22, 2, 8, 1, 4, 4, 1, 1, 0)   \
  X(23, 2, 4, 1, 2, 2, 1, 1, 0)   \
  X(24, 2, 4, 1, 4, 2, 1, 1, 0)   \
  X(25, 2, 8, 1, 4, 2, 1, 1, 0)   \
  X(26, 4, 8, 1, 1, 1, 1, 0, 0)   \
  X(27, 8, 8, 1, 1, 1, 1, 0, 0)   \
  X(28, 4, 16, 1, 1, 1, 1, 0, 0)   \
  X(29, 8, 4, 1, 1, 1, 1, 0, 0)   \
  X(30, 4, 4, 2, 4, 1, 1, 0, 0)   \
  X(31, 8, 2, 1, 2, 2, 1, 0, 0)   \
  X(32, 8, 4, 1, 2, 2, 1, 0, 0)   \
  X(33, 4, 4, 1, 2, 2, 1, 0, 0)   \
  X(34, 2, 8, 2, 2, 1, 1, 0, 0)   \
  X(35, 4, 4, 2, 2, 1, 1, 0, 0)   \
  X(36, 1, 8, 1, 2, 1, 4, 1, 1)   \
  X(37, 1, 8, 1, 1, 1, 4, 1, 1)   \
  X(38, 2, 4, 1, 2, 1, 4, 1, 0)   \
  X(39, 2, 4, 1, 1, 1, 4, 1, 0)   \
  X(40, 4, 4, 1, 1, 1, 4, 1, 0)   \
  X(41, 1, 4, 1, 2, 1, 4, 1, 1)   \
  X(42, 1, 8, 1, 2, 1, 2, 1, 1)   \
  X(43, 1, 4, 1, 4, 1, 4, 1, 0)   \
  X(44, 4, 2, 1, 2, 2, 4, 0, 0)   \
  X(45, 8, 2, 1, 2, 2, 2, 0, 0)   \
  X(46, 4, 4, 1, 1, 1, 2, 1, 0)

constexpr int kNumTiles = 47;
// Launch order: weights above kL2Resident bytes are walked one column block
// at a time over runs of kTileRun position tiles.
constexpr size_t kL2Resident = 2u << 20;
constexpr int kTileRun = 32;
constexpr size_t kMaxLds = 160 * 1024;  // LDS per workgroup on gfx950
// Complex values per thread of the register-pipelined chunk staging.
constexpr int kStageSlots = 16;
TileCfg tile_cfg(int id);
// Whether the shape has a persistent batched kernel.
bool tile_batch_ok(int id);
// Block columns of a shape.
inline int block_cols(const TileCfg& t) { return 16 * t.WC * t.FN; }
// Row fragments per wave (FM) and the LDS bytes of a wave k-split's
// reduction: each wave passes on the FM - FM / KS tiles (FN wide, 4 floats
// per lane) that other waves of its group finish.
inline int tile_fm(const TileCfg& t) { return t.T0 * t.T2 * t.WC * t.KS / 4; }
inline size_t ks_reduce_bytes(const TileCfg& t) {
  return (size_t)4 * (tile_fm(t) - tile_fm(t) / t.KS) * t.FN * 4 * 64 * sizeof(float);
}

struct ConvPlan {
  int prec;
  int tile;             // index into the shape list
  TileCfg t;
  ConvArgs a;
  int64_t gx;           // position tiles
  int gy;               // column blocks
  int run;              // position tiles per run of the launch order (see split_work)
  size_t lds_bytes;
};

// Weight layout of one contraction (shared by the weight builder and the
// convolution kernel): [chunk][k0][k1][kb][ncolp][KB], the run over
// (k2 + D - 1 taps, chunk channels, re/im) split into k-blocks of KB.
struct WeightShape {
  int chunk_c, nchunks, ps, nkb, ncolp, KB, D, cout;
  size_t elems;           // elements per part (hi or lo)
};

constexpr int kColPad = 128;  // weight columns padded to the widest block

WeightShape weight_shape(int prec, const int k[3], int cin, int chunk_c, int coutr_total, int D = 1);

// Arguments of the weight builder (one problem).
struct PrepArgs {
  const float2* F;
  int p, nc, k0, k1, k2, mode, prec;
  int chunk_c, ps, nkb, ncolp, KB, coutr_total, D;
  int64_t total;
  void* B;
  void* Blo;
};

// Build weights from the filter matrix F (n x p complex64, row-major).
//   mode 0 (forward):  input channels = coils, output columns = (filter, re/im)
//   mode 1 (adjoint):  input channels = filters, output columns = (coil, re/im),
//                      taps flipped and conjugated.
int32_t launch_prep_weights(int mode, int prec, const Geo& g, const float2* F, int p,
                            const WeightShape& ws, void* B, void* Blo, hipStream_t st);

PrepArgs make_prep_args(int mode, int prec, const Geo& g, const float2* F, int p, const WeightShape& ws, void* B,
                        void* Blo);
// One launch building the weights of `count` problems (args in device memory).
int32_t launch_prep_weights_batch(const PrepArgs* args_dev, int count, int64_t max_total, hipStream_t st);

// Default shape for a contraction with coutr real output columns (role 0
// forward / line search, 1 adjoint).
int default_tile(int prec, const Geo& g, int coutr, int role);
// Axis-2 packing a shape id implies (its D).
inline int tile_D(int id) { return tile_cfg(id).D; }

// Fill the shape-dependent fields of plan->a (everything but pointers,
// strides, org, validity box and epilogue options).  ws must be built with
// the shape's D.
int32_t plan_conv(int prec, int tile, const int k[3], const WeightShape& ws, int nchunks,
                  const int64_t oe[3], int coutr, ConvPlan* plan);

int32_t launch_conv(const ConvPlan& plan, hipStream_t st);

// Persistent launch over the work items of several problems that share one
// tile shape and precision (args and tile_start in device memory).
struct BatchConvLaunch {
  int prec;
  int tile;
  bool pipe;
  const ConvArgs* args;
  const int64_t* tile_start;
  int nprob;
  int64_t total;
  unsigned grid;
  size_t lds_bytes;
};
int32_t launch_conv_batch(const BatchConvLaunch& b, hipStream_t st);
// Whether one channel chunk of this plan fits the register staging slots.
bool conv_can_pipe(const ConvPlan& p);
// Whether the plan's tile has the compact-residual (yb != 0) variants.
bool compact_tile_ok(const ConvPlan& p);
// Widest staging unit the arguments allow: V channels of a point are read
// with 16-byte loads when the input is 16-byte aligned and the point
// stride, chunk and channel base are multiples of V.
int conv_vec(const ConvArgs& a);

// Fixed-order sum of `count` doubles into *out (single block).
int32_t launch_reduce(const double* part, int64_t count, double* out, hipStream_t st);

}  // namespace hicu
