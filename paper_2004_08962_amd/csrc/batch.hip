// Batched gradient steps for many independent problems (slices or frames of
// uneven size and coil count): one persistent launch per contraction for
// the whole batch, fixed-order per-problem reductions, and capture of a run
// of steps into one HIP graph (Algorithm 1 gradient/ELS/update steps,
// applied to every problem of the batch).
#include <algorithm>
#include <cstring>
#include <vector>

#include "batch.h"
#include "ops.h"
#include "philox.h"
#include "prof.h"
#include "step.h"
#include "tune.h"

namespace hicu {
namespace {

// Device-side per-problem tables of the small kernels.
struct JlItem {
  const float2* Q;
  float2* F;
  int n, nq, p, active;
  uint64_t seed;
};
struct RedItem {
  const double* part;
  int64_t count;
  double* out;
  const double* gnorm2;  // eta items only
};
struct UpdItem {
  float2* x;
  const float2* g;
  const double* eta;
  int64_t count;
};
struct ZeroItem {
  float2* g;
  int64_t count;
  int active;
};

// Block (j, b, q): column j, rows [64 b, 64 b + 64) of F_q = Q_q P_q with
// P_q drawn for the counter (outer, inner) read from device memory and JL
// stream id q -- the same draw and sums as the single-problem JL kernel.
__global__ __launch_bounds__(256) void jl_batch_kernel(const JlItem* items, const uint32_t* counter) {
  extern __shared__ double pcol[];
  const JlItem it = items[blockIdx.z];
  const int j = blockIdx.x, row0 = blockIdx.y * kJlRows;
  if (!it.active || j >= it.p || row0 >= it.n) return;
  jl_column_rows(it.Q, it.n, it.nq, it.p, j, row0, it.seed, counter[0], counter[1], blockIdx.z, pcol, it.F,
                 nullptr);
}

__global__ __launch_bounds__(1024) void reduce_batch_kernel(const RedItem* items) {
  __shared__ double red[16];
  const RedItem it = items[blockIdx.x];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < it.count; i += blockDim.x) s += it.part[i];
  const double tot = block_sum_d(s, red);
  if (threadIdx.x == 0) *it.out = tot;
}

__global__ __launch_bounds__(1024) void eta_batch_kernel(const RedItem* items) {
  __shared__ double red[16];
  const RedItem it = items[blockIdx.x];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < it.count; i += blockDim.x) s += it.part[i];
  const double zz = block_sum_d(s, red);
  if (threadIdx.x == 0) {
    const double gn = *it.gnorm2;
    double e = 0.0;
    if (zz > 0.0 && isfinite(zz) && isfinite(gn)) e = gn / (2.0 * zz);
    if (!isfinite(e)) e = 0.0;
    *it.out = e;
  }
}

__global__ void update_batch_kernel(const UpdItem* items) {
  const UpdItem it = items[blockIdx.y];
  const double e = *it.eta;
  if (!(e != 0.0) || !isfinite(e)) return;  // zero or non-finite step: x untouched
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < it.count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float2 gv = it.g[i];
    float2 xv = it.x[i];
    xv.x = (float)((double)xv.x - e * (double)gv.x);
    xv.y = (float)((double)xv.y - e * (double)gv.y);
    it.x[i] = xv;
  }
}

__global__ void zero_batch_kernel(const ZeroItem* items) {
  const ZeroItem it = items[blockIdx.y];
  if (!it.active) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < it.count; i += (int64_t)gridDim.x * blockDim.x)
    it.g[i] = make_float2(0.f, 0.f);
}

__global__ void counter_kernel(uint32_t* counter, uint32_t outer, uint32_t inner, int mode) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (mode == 0) {
      counter[0] = outer;
      counter[1] = inner;
    } else {
      counter[1] = counter[1] + 1u;
    }
  }
}

}  // namespace

// Per-problem plan: geometry, filters, workspace offsets.
struct BatchProblem {
  Geo g;
  int p, nq;
  bool jl;
  StepPlan sp;
  size_t off_Y, off_Bf, off_Bflo, off_Ba, off_Balo, off_pf, off_pa, off_pz, off_g, off_F;
};

}  // namespace hicu

struct hicu_batch_s {
  int count = 0, prec = 0;
  std::vector<hicu_batch_item> items;
  std::vector<hicu::BatchProblem> probs;
  int tf = 2, ta = 1;  // shape ids (batched shapes of the conv.h list)
  bool pipe_f = false, pipe_a = false;
  size_t lds_f = 0, lds_a = 0;
  int64_t total_f = 0, total_a = 0, max_prep_f = 0, max_prep_a = 0, max_n = 0, max_N = 0;
  int max_p = 0, max_nq = 0;
  bool any_zero = false, any_jl = false;
  double flops = 0.0;  // algorithmic flops of one contraction over all problems (8 n p s each)
  // algorithmic HBM bytes of the forward, adjoint and line-search launches
  double bytes_f = 0.0, bytes_a = 0.0, bytes_z = 0.0;
  // workspace layout of the shared tables
  size_t off_tables = 0, off_counter = 0, total_bytes = 0;
  size_t t_conv_f = 0, t_conv_a = 0, t_conv_z = 0, t_start_f = 0, t_start_a = 0, t_prep_f = 0, t_prep_a = 0,
         t_jl = 0, t_red_j = 0, t_red_g = 0, t_eta = 0, t_upd = 0, t_zero = 0, tables_end = 0;
  void* ws = nullptr;
  bool bound = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace hicu {

static size_t take(size_t* off, size_t bytes) {
  const size_t o = *off;
  *off += al(bytes);
  return o;
}

int32_t batch_plan(const hicu_batch_item* items, int count, int prec, hicu_batch_s* b) {
  if (prec == P_F16) return HICU_ERR_UNSUPPORTED;  // the batched path scales no operands
  b->count = count;
  b->prec = prec;
  b->items.assign(items, items + count);
  b->probs.resize(count);
  // common tile shapes: the widest column block any problem needs, 2-D or 3-D
  int ff = 1, fa = 1;
  bool any3d = false;
  for (int q = 0; q < count; ++q) {
    BatchProblem& P = b->probs[q];
    HICU_TRY(make_geo(&items[q].geom, &P.g));
    if (P.g.wrap[0] || P.g.wrap[1] || P.g.wrap[2] || P.g.kmasked)
      return HICU_ERR_UNSUPPORTED;  // circular axes, kernel masks: single-problem calls only
    if (!items[q].x || !items[q].Q || !items[q].scalars) return HICU_ERR_ARG;
    if (items[q].nq < 1 || items[q].nq >= P.g.n + 1 || items[q].p < 1 || items[q].p > items[q].nq)
      return HICU_ERR_RANK;
    P.p = items[q].p;
    P.nq = items[q].nq;
    P.jl = P.p < P.nq;
    ff = std::max<int>(ff, (int)cdiv(2 * P.p, 16));
    fa = std::max<int>(fa, (int)cdiv(2 * P.g.nc, 16));
    any3d = any3d || P.g.k[0] > 1;
  }
  // Shapes: the autotuner's batched choice (hicu_autotune_batched) for the
  // class of the problem with the most work, when it has one; else the
  // widest column block any problem needs among the batched shapes 0-2
  // (1 x 16 x 8) and 13-15 (2 x 16 x 4) with FN = 1, 2, 4.
  auto pick = [&](int frags) {
    const int fn = frags >= 3 ? 2 : frags - 1;
    return any3d ? 13 + fn : fn;
  };
  b->tf = pick(ff);
  b->ta = pick(fa);
  int chunk_a = 0;  // adjoint channel chunk from the tuner (0: first that plans of 16, 8, 4)
  {
    int big = 0;
    double wmax = -1.0;
    for (int q = 0; q < count; ++q) {
      const double w = (double)b->probs[q].g.n * b->probs[q].p * (double)b->probs[q].g.s;
      if (w > wmax) {
        wmax = w;
        big = q;
      }
    }
    TuneEntry e;
    const Geo& gb = b->probs[big].g;
    if (tune_lookup(kRoleBatchForward, prec, gb, b->probs[big].p, &e) && tile_batch_ok(e.tile) &&
        tile_D(e.tile) == 1 && (tile_cfg(e.tile).T0 == 1 || any3d))
      b->tf = e.tile;
    if (tune_lookup(kRoleBatchAdjoint, prec, gb, b->probs[big].p, &e) && tile_batch_ok(e.tile) &&
        tile_D(e.tile) == 1 && (tile_cfg(e.tile).T0 == 1 || any3d)) {
      b->ta = e.tile;
      chunk_a = e.chunk_c;
    }
  }
  size_t off = 0;
  // Register-pipelined staging pays only when a launch streams several
  // channel chunks; with one chunk per tile (up to 16 coils or filters) the
  // plain staging skips its per-slot index set-up.
  b->pipe_f = true;
  b->pipe_a = true;
  bool multi_f = false, multi_a = false;
  for (int q = 0; q < count; ++q) {
    BatchProblem& P = b->probs[q];
    const Geo& g = P.g;
    StepPlan& sp = P.sp;
    sp.wf = weight_shape(prec, g.k, g.nc, g.nc, 2 * P.p, 1);
    int32_t s = plan_conv(prec, b->tf, g.k, sp.wf, sp.wf.nchunks, g.m, 2 * P.p, &sp.cf);
    if (s != HICU_OK) return s;
    const int64_t oe[3] = {g.hi[0] - g.lo[0], g.hi[1] - g.lo[1], g.hi[2] - g.lo[2]};
    s = HICU_ERR_UNSUPPORTED;
    for (int cc : {16, 8, 4}) {
      const int c = chunk_a > 0 ? chunk_a : cc;
      sp.wa = weight_shape(prec, g.k, P.p, std::min(c, P.p), 2 * g.nc, 1);
      s = plan_conv(prec, b->ta, g.k, sp.wa, sp.wa.nchunks, oe, 2 * g.nc, &sp.ca);
      if (s != HICU_ERR_UNSUPPORTED) break;
      chunk_a = 0;  // the tuned chunk does not plan for this problem: fall back
    }
    if (s != HICU_OK) return s;
    sp.nf_blocks = sp.cf.gx * sp.cf.gy;
    sp.na_blocks = sp.ca.gx * sp.ca.gy;
    b->pipe_f = b->pipe_f && conv_can_pipe(sp.cf);
    b->pipe_a = b->pipe_a && conv_can_pipe(sp.ca);
    multi_f = multi_f || sp.cf.a.nchunks > 1;
    multi_a = multi_a || sp.ca.a.nchunks > 1;
    b->lds_f = std::max(b->lds_f, sp.cf.lds_bytes);
    b->lds_a = std::max(b->lds_a, sp.ca.lds_bytes);
    b->total_f += sp.nf_blocks;
    b->total_a += sp.na_blocks;
    b->max_prep_f = std::max<int64_t>(b->max_prep_f, (int64_t)sp.wf.elems);
    b->max_prep_a = std::max<int64_t>(b->max_prep_a, (int64_t)sp.wa.elems);
    const int64_t N = g.npts * g.nc;
    b->max_N = std::max(b->max_N, N);
    b->max_n = std::max<int64_t>(b->max_n, g.n);
    b->max_p = std::max(b->max_p, P.p);
    b->max_nq = std::max(b->max_nq, P.nq);
    b->any_zero = b->any_zero || !full_region(g);
    b->any_jl = b->any_jl || P.jl;
    b->flops += 8.0 * g.n * (double)P.p * (double)g.s;
    const double nS = (double)region_points(g), ys = 8.0 * (double)g.s * P.p;
    b->bytes_f += 8.0 * nS * g.nc + ys;
    b->bytes_a += ys + nS + 8.0 * nS * g.nc;
    b->bytes_z += 8.0 * nS * g.nc;
    const size_t es = esize(prec), parts = prec == P_BF16X3 ? 2 : 1;
    P.off_Y = take(&off, (size_t)g.s * P.p * sizeof(float2));
    P.off_Bf = take(&off, sp.wf.elems * es);
    P.off_Bflo = parts > 1 ? take(&off, sp.wf.elems * es) : P.off_Bf;
    P.off_Ba = take(&off, sp.wa.elems * es);
    P.off_Balo = parts > 1 ? take(&off, sp.wa.elems * es) : P.off_Ba;
    P.off_pf = take(&off, sp.nf_blocks * sizeof(double));
    P.off_pa = take(&off, sp.na_blocks * sizeof(double));
    P.off_pz = take(&off, sp.nf_blocks * sizeof(double));
    P.off_g = take(&off, (size_t)N * sizeof(float2));
    P.off_F = take(&off, P.jl ? (size_t)g.n * P.p * sizeof(float2) : 0);
  }
  b->pipe_f = b->pipe_f && multi_f;
  b->pipe_a = b->pipe_a && multi_a;
  if ((size_t)b->max_nq * sizeof(double) > 65536) return HICU_ERR_UNSUPPORTED;
  b->off_tables = off;
  b->t_conv_f = take(&off, count * sizeof(ConvArgs));
  b->t_conv_a = take(&off, count * sizeof(ConvArgs));
  b->t_conv_z = take(&off, count * sizeof(ConvArgs));
  b->t_start_f = take(&off, (count + 1) * sizeof(int64_t));
  b->t_start_a = take(&off, (count + 1) * sizeof(int64_t));
  b->t_prep_f = take(&off, count * sizeof(PrepArgs));
  b->t_prep_a = take(&off, count * sizeof(PrepArgs));
  b->t_jl = take(&off, count * sizeof(JlItem));
  b->t_red_j = take(&off, count * sizeof(RedItem));
  b->t_red_g = take(&off, count * sizeof(RedItem));
  b->t_eta = take(&off, count * sizeof(RedItem));
  b->t_upd = take(&off, count * sizeof(UpdItem));
  b->t_zero = take(&off, count * sizeof(ZeroItem));
  b->tables_end = off;
  b->off_counter = take(&off, 4 * sizeof(uint32_t));
  b->total_bytes = off;
  return HICU_OK;
}

int32_t batch_bind(hicu_batch_s* b, void* ws, hipStream_t st) {
  const int count = b->count, prec = b->prec;
  std::vector<ConvArgs> cf(count), ca(count), cz(count);
  std::vector<int64_t> sf(count + 1), sa(count + 1);
  std::vector<PrepArgs> pf(count), pa(count);
  std::vector<JlItem> jl(count);
  std::vector<RedItem> rj(count), rg(count), re(count);
  std::vector<UpdItem> up(count);
  std::vector<ZeroItem> zr(count);
  sf[0] = sa[0] = 0;
  for (int q = 0; q < count; ++q) {
    BatchProblem& P = b->probs[q];
    const hicu_batch_item& it = b->items[q];
    const Geo& g = P.g;
    StepPlan& sp = P.sp;
    const float2* F = P.jl ? reinterpret_cast<const float2*>(at(ws, P.off_F)) : reinterpret_cast<const float2*>(it.Q);
    double* sc = it.scalars;
    float2* gq = reinterpret_cast<float2*>(at(ws, P.off_g));
    sp.off_Bf = P.off_Bf;
    sp.off_Bflo = P.off_Bflo;
    // forward: x -> Y, partials pf
    fill_forward_args(g, it.x, sp, ws, reinterpret_cast<float*>(at(ws, P.off_Y)),
                      reinterpret_cast<double*>(at(ws, P.off_pf)));
    cf[q] = sp.cf.a;
    cf[q].vec = conv_vec(cf[q]);
    // line search: g -> (no output), partials pz
    fill_forward_args(g, gq, sp, ws, nullptr, reinterpret_cast<double*>(at(ws, P.off_pz)));
    cz[q] = sp.cf.a;
    cz[q].vec = conv_vec(cz[q]);
    // adjoint: Y -> g, partials pa
    fill_adjoint_args(g, at(ws, P.off_Y), P.p, at(ws, P.off_Ba), at(ws, P.off_Balo), gq, it.mask,
                      reinterpret_cast<double*>(at(ws, P.off_pa)), sp.ca.a);
    ca[q] = sp.ca.a;
    ca[q].vec = conv_vec(ca[q]);
    // pipelined staging moves four aligned channels per slot
    if (cf[q].vec != 4 || cz[q].vec != 4) b->pipe_f = false;
    if (ca[q].vec != 4) b->pipe_a = false;
    sf[q + 1] = sf[q] + sp.nf_blocks;
    sa[q + 1] = sa[q] + sp.na_blocks;
    pf[q] = make_prep_args(0, prec, g, F, P.p, sp.wf, at(ws, P.off_Bf), at(ws, P.off_Bflo));
    pa[q] = make_prep_args(1, prec, g, F, P.p, sp.wa, at(ws, P.off_Ba), at(ws, P.off_Balo));
    jl[q] = JlItem{reinterpret_cast<const float2*>(it.Q), reinterpret_cast<float2*>(at(ws, P.off_F)), g.n, P.nq,
                   P.p, P.jl ? 1 : 0, it.seed};
    rj[q] = RedItem{reinterpret_cast<const double*>(at(ws, P.off_pf)), sp.nf_blocks, sc + 0, nullptr};
    rg[q] = RedItem{reinterpret_cast<const double*>(at(ws, P.off_pa)), sp.na_blocks, sc + 1, nullptr};
    re[q] = RedItem{reinterpret_cast<const double*>(at(ws, P.off_pz)), sp.nf_blocks, sc + 2, sc + 1};
    up[q] = UpdItem{reinterpret_cast<float2*>(it.x), gq, sc + 2, g.npts * g.nc};
    zr[q] = ZeroItem{gq, g.npts * g.nc, full_region(g) ? 0 : 1};
  }
  auto put = [&](size_t off, const void* src, size_t bytes) {
    return hipMemcpyAsync(at(ws, off), src, bytes, hipMemcpyHostToDevice, st);
  };
  HICU_HIP_TRY(put(b->t_conv_f, cf.data(), count * sizeof(ConvArgs)));
  HICU_HIP_TRY(put(b->t_conv_a, ca.data(), count * sizeof(ConvArgs)));
  HICU_HIP_TRY(put(b->t_conv_z, cz.data(), count * sizeof(ConvArgs)));
  HICU_HIP_TRY(put(b->t_start_f, sf.data(), (count + 1) * sizeof(int64_t)));
  HICU_HIP_TRY(put(b->t_start_a, sa.data(), (count + 1) * sizeof(int64_t)));
  HICU_HIP_TRY(put(b->t_prep_f, pf.data(), count * sizeof(PrepArgs)));
  HICU_HIP_TRY(put(b->t_prep_a, pa.data(), count * sizeof(PrepArgs)));
  HICU_HIP_TRY(put(b->t_jl, jl.data(), count * sizeof(JlItem)));
  HICU_HIP_TRY(put(b->t_red_j, rj.data(), count * sizeof(RedItem)));
  HICU_HIP_TRY(put(b->t_red_g, rg.data(), count * sizeof(RedItem)));
  HICU_HIP_TRY(put(b->t_eta, re.data(), count * sizeof(RedItem)));
  HICU_HIP_TRY(put(b->t_upd, up.data(), count * sizeof(UpdItem)));
  HICU_HIP_TRY(put(b->t_zero, zr.data(), count * sizeof(ZeroItem)));
  hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(at(ws, b->off_counter)),
                     0u, 0u, 0);
  HICU_HIP_TRY(hipGetLastError());
  HICU_HIP_TRY(hipStreamSynchronize(st));  // host vectors go out of scope
  b->ws = ws;
  b->bound = true;
  return HICU_OK;
}

// One gradient step (JL draw, weights, forward + J, adjoint + ||g||^2, line
// search, update) for every problem: kernel launches only.
int32_t batch_step(hicu_batch_s* b, hipStream_t st) {
  void* ws = b->ws;
  const int count = b->count;
  // persistent workgroups per contraction launch: measured on 64 uneven
  // 2-D slices, 8192 ran the BF16 step 8 % faster than 2048 (16384 and one
  // workgroup per item were slower again)
  const unsigned grid = 8192;
  uint32_t* counter = reinterpret_cast<uint32_t*>(at(ws, b->off_counter));
  if (b->any_jl) {
    ProfScope ps("jl", st);
    hipLaunchKernelGGL(jl_batch_kernel, dim3(b->max_p, (unsigned)cdiv(b->max_n, kJlRows), count), dim3(256),
                       b->max_nq * sizeof(double), st, reinterpret_cast<const JlItem*>(at(ws, b->t_jl)),
                       (const uint32_t*)counter);
  }
  {
    ProfScope ps("prep_weights", st, 0.0, 0.0, true);
    HICU_TRY(launch_prep_weights_batch(reinterpret_cast<const PrepArgs*>(at(ws, b->t_prep_f)), count, b->max_prep_f,
                                       st));
    HICU_TRY(launch_prep_weights_batch(reinterpret_cast<const PrepArgs*>(at(ws, b->t_prep_a)), count, b->max_prep_a,
                                       st));
  }
  BatchConvLaunch f{b->prec, b->tf, b->pipe_f, reinterpret_cast<const ConvArgs*>(at(ws, b->t_conv_f)),
                    reinterpret_cast<const int64_t*>(at(ws, b->t_start_f)), count, b->total_f,
                    (unsigned)std::min<int64_t>(grid, b->total_f), b->lds_f};
  {
    ProfScope ps("batch_conv_fwd", st, b->flops, b->bytes_f);
    HICU_TRY(launch_conv_batch(f, st));
  }
  hipLaunchKernelGGL(reduce_batch_kernel, dim3(count), dim3(1024), 0, st,
                     reinterpret_cast<const RedItem*>(at(ws, b->t_red_j)));
  if (b->any_zero) {
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(b->max_N, 256), 1024));
    hipLaunchKernelGGL(zero_batch_kernel, dim3((unsigned)blocks, count), dim3(256), 0, st,
                       reinterpret_cast<const ZeroItem*>(at(ws, b->t_zero)));
  }
  BatchConvLaunch a{b->prec, b->ta, b->pipe_a, reinterpret_cast<const ConvArgs*>(at(ws, b->t_conv_a)),
                    reinterpret_cast<const int64_t*>(at(ws, b->t_start_a)), count, b->total_a,
                    (unsigned)std::min<int64_t>(grid, b->total_a), b->lds_a};
  {
    ProfScope ps("batch_conv_adj", st, b->flops, b->bytes_a);
    HICU_TRY(launch_conv_batch(a, st));
  }
  hipLaunchKernelGGL(reduce_batch_kernel, dim3(count), dim3(1024), 0, st,
                     reinterpret_cast<const RedItem*>(at(ws, b->t_red_g)));
  BatchConvLaunch z = f;
  z.args = reinterpret_cast<const ConvArgs*>(at(ws, b->t_conv_z));
  {
    ProfScope ps("batch_conv_els", st, b->flops, b->bytes_z);
    HICU_TRY(launch_conv_batch(z, st));
  }
  hipLaunchKernelGGL(eta_batch_kernel, dim3(count), dim3(1024), 0, st,
                     reinterpret_cast<const RedItem*>(at(ws, b->t_eta)));
  {
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(b->max_N, 256), 1024));
    hipLaunchKernelGGL(update_batch_kernel, dim3((unsigned)blocks, count), dim3(256), 0, st,
                       reinterpret_cast<const UpdItem*>(at(ws, b->t_upd)));
  }
  if (b->any_jl) hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, st, counter, 0u, 0u, 1);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

}  // namespace hicu

using namespace hicu;

extern "C" {

int32_t hicu_batch_create(const hicu_batch_item* items, int32_t count, int32_t prec, hicu_batch** out,
                          size_t* ws_bytes) {
  if (!items || !out || count < 1 || count > 65535 || !valid_prec(prec)) return HICU_ERR_ARG;
  hicu_batch_s* b = new (std::nothrow) hicu_batch_s();
  if (!b) return HICU_ERR_ARG;
  const int32_t s = batch_plan(items, count, prec, b);
  if (s != HICU_OK) {
    delete b;
    return s;
  }
  if (ws_bytes) *ws_bytes = b->total_bytes;
  *out = b;
  return HICU_OK;
}

int32_t hicu_batch_bind(hicu_batch* b, void* ws, size_t ws_bytes, void* stream) {
  if (!b || !ws) return HICU_ERR_ARG;
  if (ws_bytes < b->total_bytes) return HICU_ERR_WORKSPACE;
  return batch_bind(b, ws, (hipStream_t)stream);
}

int32_t hicu_batch_set_counter(hicu_batch* b, uint32_t outer, uint32_t inner, void* stream) {
  if (!b || !b->bound) return HICU_ERR_ARG;
  hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream,
                     reinterpret_cast<uint32_t*>(at(b->ws, b->off_counter)), outer, inner, 0);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

int32_t hicu_batch_step(hicu_batch* b, void* stream) {
  if (!b || !b->bound) return HICU_ERR_ARG;
  return batch_step(b, (hipStream_t)stream);
}

int32_t hicu_batch_graph_create(hicu_batch* b, int32_t steps, void* stream) {
  if (!b || !b->bound || steps < 1 || !stream) return HICU_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  HICU_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  int32_t s = HICU_OK;
  for (int i = 0; i < steps && s == HICU_OK; ++i) s = batch_step(b, st);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  if (s != HICU_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return HICU_ERR_HIP;
  b->graph = g;
  HICU_HIP_TRY(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  return HICU_OK;
}

int32_t hicu_batch_graph_launch(hicu_batch* b, void* stream) {
  if (!b || !b->exec) return HICU_ERR_ARG;
  HICU_HIP_TRY(hipGraphLaunch(b->exec, (hipStream_t)stream));
  return HICU_OK;
}

int32_t hicu_batch_info(const hicu_batch* b, int64_t* info) {
  if (!b || !info) return HICU_ERR_ARG;
  info[0] = b->count;
  info[1] = b->total_f;
  info[2] = b->total_a;
  info[3] = b->tf;
  info[4] = b->ta;
  info[5] = (int64_t)b->total_bytes;
  return HICU_OK;
}

void hicu_batch_destroy(hicu_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  delete b;
}

}  // extern "C"
