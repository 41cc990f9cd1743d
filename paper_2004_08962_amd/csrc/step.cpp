// Planning and launch sequence of one gradient step (objective, gradient,
// exact line search) for one problem; shared by the C entry points, the
// solver loop and the batched runtime.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "ops.h"
#include "prof.h"
#include "step.h"
#include "tune.h"

namespace hicu {


int32_t plan_forward(const Geo& g, int p, int prec, WeightShape* w, ConvPlan* c) {
  TuneEntry e;
  if (tune_lookup(0, prec, g, p, &e) && tile_D(e.tile) == 1) {
    *w = weight_shape(prec, g.k, g.nc, g.nc, 2 * p, 1);
    if (plan_conv(prec, e.tile, g.k, *w, w->nchunks, g.m, 2 * p, c) == HICU_OK) return HICU_OK;
  }
  *w = weight_shape(prec, g.k, g.nc, g.nc, 2 * p, 1);
  int32_t s = plan_conv(prec, default_tile(prec, g, 2 * p, 0), g.k, *w, w->nchunks, g.m, 2 * p, c);
  if (s == HICU_ERR_UNSUPPORTED) s = plan_conv(prec, 0, g.k, *w, w->nchunks, g.m, 2 * p, c);
  return s;
}

int32_t plan_adjoint(const Geo& g, int p, int prec, WeightShape* w, ConvPlan* c) {
  const int64_t oe[3] = {g.hi[0] - g.lo[0], g.hi[1] - g.lo[1], g.hi[2] - g.lo[2]};
  TuneEntry e;
  if (tune_lookup(1, prec, g, p, &e)) {
    *w = weight_shape(prec, g.k, p, std::min(e.chunk_c, std::max(1, p)), 2 * g.nc, tile_D(e.tile));
    if (plan_conv(prec, e.tile, g.k, *w, w->nchunks, oe, 2 * g.nc, c) == HICU_OK) return HICU_OK;
  }
  int32_t s = HICU_ERR_UNSUPPORTED;
  const int tiles[2] = {default_tile(prec, g, 2 * g.nc, 1), 0};
  // volumes stage 8 channels per chunk (a 6 x 20 x 12 halo), planes 16
  const int order3[5] = {8, 16, 4, 2, 1}, order2[5] = {16, 8, 4, 2, 1};
  const int* order = g.k[0] > 1 ? order3 : order2;
  for (const int t : tiles) {
    for (int oi = 0; oi < 5; ++oi) {
      const int cc = order[oi];
      *w = weight_shape(prec, g.k, p, std::min(cc, std::max(1, p)), 2 * g.nc, tile_D(t));
      s = plan_conv(prec, t, g.k, *w, w->nchunks, oe, 2 * g.nc, c);
      if (s != HICU_ERR_UNSUPPORTED) return s;
    }
  }
  return s;
}

static std::atomic<size_t> y_budget{kYBudget};

void set_y_budget(size_t bytes) { y_budget.store(bytes ? bytes : kYBudget); }

int filter_group(int64_t s, int p, size_t bytes) {
  const size_t per = (size_t)std::max<int64_t>(s, 1) * bytes;
  const size_t budget = y_budget.load();
  if ((size_t)p * per <= budget) return p;
  return (int)std::min<size_t>((size_t)p, std::max<size_t>(64, budget / per / 64 * 64));
}

// Column blocks of the forward launch restricted to filters [c0, c0 + pg).
static int group_col_blocks(const ConvPlan& c, int pg) { return (int)cdiv(2 * pg, block_cols(c.t)); }

int32_t make_step_plan(const Geo& g, int p, int prec, bool need_adj, StepPlan* sp) {
  HICU_TRY(plan_forward(g, p, prec, &sp->wf, &sp->cf));
  if (need_adj) HICU_TRY(plan_adjoint(g, p, prec, &sp->wa, &sp->ca));
  sp->pc = need_adj ? filter_group(g.s, p) : p;
  // When Y does not fit at once (filter groups), the BF16 path stores it as
  // BF16: the adjoint rounds its operand to BF16 anyway, so the stored
  // values are the ones it would stage, at half the bytes to write and
  // re-read.  Blocks of the adjoint's chunk width keep every chunk's staging
  // reads contiguous.
  sp->ybw = 0;
  if (need_adj && sp->pc < p && compact_tile_ok(sp->cf) && compact_tile_ok(sp->ca)) {
    sp->ybw = sp->ca.a.chunk_c;
    sp->pc = filter_group(g.s, p, sizeof(uint32_t));
  }
  // Forward partial sums: one per (tile, column block) of every filter group.
  int64_t gy = 0;
  for (int c0 = 0; c0 < p; c0 += sp->pc) gy += group_col_blocks(sp->cf, std::min(sp->pc, p - c0));
  sp->nf_blocks = sp->cf.gx * std::max<int64_t>(gy, sp->cf.gy);
  sp->na_blocks = 0;
  size_t off = 0;
  sp->off_Y = off;
  if (need_adj)
    off += al(sp->ybw ? (size_t)g.s * rup(sp->pc, sp->ybw) * sizeof(uint32_t) : (size_t)g.s * sp->pc * sizeof(float2));
  sp->off_Bf = off;
  off += al(sp->wf.elems * esize(prec));
  sp->off_Bflo = off;
  if (prec == P_BF16X3) off += al(sp->wf.elems * esize(prec));
  sp->off_Ba = sp->off_Balo = off;
  if (need_adj) {
    sp->na_blocks = sp->ca.gx * sp->ca.gy;
    sp->off_Ba = off;
    off += al(sp->wa.elems * esize(prec));
    sp->off_Balo = off;
    if (prec == P_BF16X3) off += al(sp->wa.elems * esize(prec));
  }
  sp->off_pf = off;
  off += al(sp->nf_blocks * sizeof(double));
  sp->off_pa = off;
  off += al(std::max<int64_t>(1, sp->na_blocks) * sizeof(double));
  sp->off_pz = off;
  off += al(sp->nf_blocks * sizeof(double));
  // FP16 operand scales (x, Y, g) and per-block maxima
  sp->off_sc = off;
  off += al(4 * sizeof(float));
  sp->off_pmax = off;
  off += al(std::max<int64_t>(kAbsmaxBlocks, sp->nf_blocks) * sizeof(float));
  sp->total = off;
  return HICU_OK;
}

// Profiler tag of a contraction: kind (0 forward, 1 adjoint, 2 line search) x precision.
const char* conv_tag(int kind, int prec) {
  static const char* tags[3][4] = {{"conv_fwd_fp32", "conv_fwd_bf16", "conv_fwd_bf16x3", "conv_fwd_fp16"},
                                   {"conv_adj_fp32", "conv_adj_bf16", "conv_adj_bf16x3", "conv_adj_fp16"},
                                   {"conv_els_fp32", "conv_els_bf16", "conv_els_bf16x3", "conv_els_fp16"}};
  return tags[kind][prec];
}


int64_t region_points(const Geo& g) {
  return (g.hi[0] - g.lo[0]) * (g.hi[1] - g.lo[1]) * (g.hi[2] - g.lo[2]);
}

bool full_region(const Geo& g) {
  for (int a = 0; a < 3; ++a)
    if (g.lo[a] != 0 || g.hi[a] != g.d[a]) return false;
  return true;
}

void fill_forward_args(const Geo& g, const void* in, StepPlan& sp, void* ws, float* out, double* partial) {
  ConvArgs& a = sp.cf.a;
  a.in = reinterpret_cast<const float2*>(in);
  a.is[0] = g.d[1] * g.d[2] * g.nc;
  a.is[1] = g.d[2] * g.nc;
  a.is[2] = g.nc;
  a.cin = g.nc;
  a.chan_base = 0;
  a.ch0 = 0;
  for (int i = 0; i < 3; ++i) {
    a.vlo[i] = 0;
    a.vhi[i] = g.d[i];
    a.org[i] = g.lo[i];
    a.wp[i] = g.wrap[i] ? g.d[i] : 0;
  }
  a.B = at(ws, sp.off_Bf);
  a.Blo = at(ws, sp.off_Bflo);
  a.col0 = 0;
  a.out = out;
  const int p = sp.cf.a.coutr / 2;
  a.os[0] = g.m[1] * g.m[2] * p;
  a.os[1] = g.m[2] * p;
  a.os[2] = p;
  a.mask = nullptr;
  for (int i = 0; i < 3; ++i) {
    a.ms[i] = 0;
    a.morg[i] = 0;
  }
  a.scale = 1.f;
  a.accumulate = 0;
  a.partial = partial;
  a.in_scale = nullptr;
  a.absmax = nullptr;
}

void fill_adjoint_args(const Geo& g, const void* Y, int p, const void* B, const void* Blo, void* gout,
                       const uint8_t* mask, double* partial, ConvArgs& a) {
  a.in = reinterpret_cast<const float2*>(Y);
  a.is[0] = g.m[1] * g.m[2] * p;
  a.is[1] = g.m[2] * p;
  a.is[2] = p;
  a.cin = p;
  a.chan_base = 0;
  a.ch0 = 0;
  for (int i = 0; i < 3; ++i) {
    a.vlo[i] = 0;
    a.vhi[i] = g.m[i];
    a.org[i] = -(int64_t)(g.k[i] - 1);
    a.wp[i] = g.wrap[i] ? g.m[i] : 0;
  }
  a.B = B;
  a.Blo = Blo;
  a.col0 = 0;
  const int64_t base = ((g.lo[0] * g.d[1] + g.lo[1]) * g.d[2] + g.lo[2]) * g.nc;
  a.out = reinterpret_cast<float*>(reinterpret_cast<float2*>(gout) + base);
  a.os[0] = g.d[1] * g.d[2] * g.nc;
  a.os[1] = g.d[2] * g.nc;
  a.os[2] = g.nc;
  a.mask = mask;
  a.ms[0] = g.d[1] * g.d[2];
  a.ms[1] = g.d[2];
  a.ms[2] = 1;
  for (int i = 0; i < 3; ++i) a.morg[i] = g.lo[i];
  a.scale = 2.f;
  a.accumulate = 0;
  a.partial = partial;
  a.in_scale = nullptr;
  a.absmax = nullptr;
}

// Objective, gradient; shared by the public entry and the solver loop.
// Filters are taken in groups of sp.pc: the forward launch of a group writes
// its columns of Y = H_S(x)F (and its share of the sum of squares), the
// adjoint launch of the group adds H_S'(Y_group F_group^H) into g.  The sum
// over groups is the full adjoint because H_S'(Y F^H) is linear in the
// filter columns; the last group writes the per-block sums of |g|^2.
// Kernel masks: the filters are spread to the whole box (zero rows outside
// the mask) at the head of the workspace and the step runs on the box.
static size_t kmask_head(const Geo& g, int p) { return g.kmasked ? al((size_t)g.nbox * p * sizeof(float2)) : 0; }

int32_t objective_grad_impl(const Geo& g, const void* x, const uint8_t* mask, const void* F, int p, int prec,
                            double* J, void* gout, double* gn2, void* ws, size_t ws_bytes, hipStream_t st,
                            int prep) {
  if (g.kmasked) {
    const size_t h = kmask_head(g, p);
    if (!ws || ws_bytes < h) return HICU_ERR_WORKSPACE;
    if (prep) HICU_TRY(launch_kmask_scatter(g, reinterpret_cast<const float2*>(F), p, reinterpret_cast<float2*>(ws), st));
    return objective_grad_impl(box_geo(g), x, mask, ws, p, prec, J, gout, gn2, at(ws, h), ws_bytes - h, st, prep);
  }
  StepPlan sp;
  HICU_TRY(make_step_plan(g, p, prec, gout != nullptr, &sp));
  if (!ws || ws_bytes < sp.total) return HICU_ERR_WORKSPACE;
  const float2* Fc = reinterpret_cast<const float2*>(F);
  const double nS = (double)region_points(g);
  if (prep & kPrepForward) {
    ProfScope ps("prep_weights", st, 0.0, 0.0, true);
    HICU_TRY(launch_prep_weights(0, prec, g, Fc, p, sp.wf, at(ws, sp.off_Bf), at(ws, sp.off_Bflo), st));
  }
  float2* Y = reinterpret_cast<float2*>(at(ws, sp.off_Y));
  double* pf = reinterpret_cast<double*>(at(ws, sp.off_pf));
  double* pa = reinterpret_cast<double*>(at(ws, sp.off_pa));
  // FP16: scale of x from its largest magnitude; per group, scale of Y from
  // the forward's per-block maxima
  const bool f16 = prec == P_F16;
  float* scales = reinterpret_cast<float*>(at(ws, sp.off_sc));
  float* pmax = reinterpret_cast<float*>(at(ws, sp.off_pmax));
  if (f16) {
    ProfScope ps("scale", st, 0.0, 0.0, true);
    HICU_TRY(launch_absmax(reinterpret_cast<const float*>(x), 2 * g.npts * g.nc, pmax, st));
    HICU_TRY(launch_scale(pmax, kAbsmaxBlocks, scales, st));
  }
  if (gout) {
    if (!full_region(g)) {
      ProfScope ps("zero", st, 0.0, 0.0, true);
      HICU_TRY(launch_zero(gout, (size_t)g.npts * g.nc * sizeof(float2), st));
    }
    if (prep & kPrepAdjoint) {
      ProfScope ps("prep_weights", st, 0.0, 0.0, true);
      HICU_TRY(launch_prep_weights(1, prec, g, Fc, p, sp.wa, at(ws, sp.off_Ba), at(ws, sp.off_Balo), st));
    }
  }
  int64_t pf_used = 0;
  const double ybytes = sp.ybw ? 4.0 : 8.0;  // bytes per stored residual value
  for (int c0 = 0; c0 < p; c0 += sp.pc) {
    const int pg = std::min(sp.pc, p - c0);
    const bool last = c0 + pg == p;
    const double flops = 8.0 * g.n * (double)pg * (double)g.s;
    ConvPlan cf = sp.cf;
    fill_forward_args(g, x, sp, ws, gout ? reinterpret_cast<float*>(Y) : nullptr, pf + pf_used);
    cf.a = sp.cf.a;
    cf.a.col0 = 2 * c0;
    cf.a.coutr = 2 * pg;
    cf.gy = group_col_blocks(cf, pg);
    if (sp.ybw) {  // compact BF16 Y: blocks of ybw filters, points strided by ybw inside a block
      cf.a.yb = 2;
      cf.a.ybw = sp.ybw;
      cf.a.yblk = g.s * sp.ybw;
      cf.a.os[0] = g.m[1] * g.m[2] * sp.ybw;
      cf.a.os[1] = g.m[2] * sp.ybw;
      cf.a.os[2] = sp.ybw;
    } else {
      cf.a.os[0] = g.m[1] * g.m[2] * pg;
      cf.a.os[1] = g.m[2] * pg;
      cf.a.os[2] = pg;
    }
    if (f16) {
      cf.a.in_scale = scales;
      if (gout) cf.a.absmax = pmax + pf_used;
    }
    const int64_t pmax0 = pf_used;
    pf_used += cf.gx * cf.gy;
    {
      ProfScope ps(conv_tag(0, prec), st, flops, 8.0 * nS * g.nc + (gout ? ybytes * (double)g.s * pg : 0.0));
      HICU_TRY(launch_conv(cf, st));
    }
    if (!gout) continue;
    ConvPlan ca = sp.ca;
    fill_adjoint_args(g, Y, pg, at(ws, sp.off_Ba), at(ws, sp.off_Balo), gout, mask, last ? pa : nullptr, ca.a);
    ca.a.cin = c0 + pg;
    ca.a.chan_base = c0;
    ca.a.ch0 = c0 / ca.a.chunk_c;
    ca.a.nchunks = (int)cdiv(pg, ca.a.chunk_c);
    ca.a.accumulate = c0 > 0;
    if (sp.ybw) {
      ca.a.yb = 1;
      ca.a.ybw = sp.ybw;
      ca.a.yblk = g.s * sp.ybw;
      ca.a.is[0] = g.m[1] * g.m[2] * sp.ybw;
      ca.a.is[1] = g.m[2] * sp.ybw;
      ca.a.is[2] = sp.ybw;
    }
    if (f16) {
      ProfScope ps("scale", st, 0.0, 0.0, true);
      HICU_TRY(launch_scale(pmax + pmax0, cf.gx * cf.gy, scales + 1, st));
      ca.a.in_scale = scales + 1;
    }
    {
      ProfScope ps(conv_tag(1, prec), st, flops, ybytes * (double)g.s * pg + 8.0 * nS * g.nc * (c0 > 0 ? 2 : 1) + nS);
      HICU_TRY(launch_conv(ca, st));
    }
  }
  if (J) {
    ProfScope ps("reduce", st, 0.0, 0.0, true);
    HICU_TRY(launch_reduce(pf, pf_used, J, st));
  }
  if (gout && gn2) {
    ProfScope ps("reduce", st, 0.0, 0.0, true);
    HICU_TRY(launch_reduce(pa, sp.na_blocks, gn2, st));
  }
  return HICU_OK;
}

int32_t line_search_impl(const Geo& g, const void* gv, const double* gn2, const void* F, int p, int prec,
                         double* eta, void* ws, size_t ws_bytes, hipStream_t st, bool grad_weights) {
  if (g.kmasked) {
    const size_t h = kmask_head(g, p);
    if (!ws || ws_bytes < h) return HICU_ERR_WORKSPACE;
    if (!grad_weights)
      HICU_TRY(launch_kmask_scatter(g, reinterpret_cast<const float2*>(F), p, reinterpret_cast<float2*>(ws), st));
    return line_search_impl(box_geo(g), gv, gn2, ws, p, prec, eta, at(ws, h), ws_bytes - h, st, grad_weights);
  }
  StepPlan sp;
  HICU_TRY(make_step_plan(g, p, prec, false, &sp));
  // The line-search layout is a prefix-compatible subset of the gradient
  // layout only when no Y is stored, so it has its own offsets.  With
  // grad_weights the forward weights that objective_grad_impl prepared for
  // the same F, precision and geometry are read where the gradient layout
  // put them (the forward plan is the same in both layouts).
  if (grad_weights) {
    StepPlan gp;
    HICU_TRY(make_step_plan(g, p, prec, true, &gp));
    if (!ws || ws_bytes < gp.total) return HICU_ERR_WORKSPACE;
    sp.off_Bf = gp.off_Bf;
    sp.off_Bflo = gp.off_Bflo;
    sp.off_pz = gp.off_pz;
    sp.off_sc = gp.off_sc;
    sp.off_pmax = gp.off_pmax;
  }
  if (!ws || ws_bytes < sp.total) return HICU_ERR_WORKSPACE;
  if (!grad_weights) {
    ProfScope ps("prep_weights", st, 0.0, 0.0, true);
    HICU_TRY(launch_prep_weights(0, prec, g, reinterpret_cast<const float2*>(F), p, sp.wf, at(ws, sp.off_Bf),
                                 at(ws, sp.off_Bflo), st));
  }
  double* pz = reinterpret_cast<double*>(at(ws, sp.off_pz));
  fill_forward_args(g, gv, sp, ws, nullptr, pz);
  if (prec == P_F16) {
    ProfScope ps("scale", st, 0.0, 0.0, true);
    float* scales = reinterpret_cast<float*>(at(ws, sp.off_sc));
    float* pmax = reinterpret_cast<float*>(at(ws, sp.off_pmax));
    HICU_TRY(launch_absmax(reinterpret_cast<const float*>(gv), 2 * g.npts * g.nc, pmax, st));
    HICU_TRY(launch_scale(pmax, kAbsmaxBlocks, scales + 2, st));
    sp.cf.a.in_scale = scales + 2;
  }
  {
    ProfScope ps(conv_tag(2, prec), st, 8.0 * g.n * (double)p * (double)g.s, 8.0 * (double)region_points(g) * g.nc);
    HICU_TRY(launch_conv(sp.cf, st));
  }
  {
    ProfScope ps("eta", st, 0.0, 0.0, true);
    HICU_TRY(launch_eta(pz, sp.nf_blocks, gn2, eta, st));
  }
  return HICU_OK;
}

// Y = H_S(x) F kept whole (s x p complex64, point-major, filter fastest):
// the sketch of the randomized SVD.  One forward launch over all p filters.
size_t forward_store_workspace(const Geo& g, int p, int prec) {
  if (g.kmasked) {
    const size_t inner = forward_store_workspace(box_geo(g), p, prec);
    return inner ? kmask_head(g, p) + inner : 0;
  }
  StepPlan sp;
  if (make_step_plan(g, p, prec, false, &sp) != HICU_OK) return 0;
  return sp.total;
}

int32_t forward_store_impl(const Geo& g, const void* x, const void* F, int p, int prec, void* Y, void* ws,
                           size_t ws_bytes, hipStream_t st) {
  if (prec == P_F16) return HICU_ERR_UNSUPPORTED;
  if (g.kmasked) {
    const size_t h = kmask_head(g, p);
    if (!ws || ws_bytes < h) return HICU_ERR_WORKSPACE;
    HICU_TRY(launch_kmask_scatter(g, reinterpret_cast<const float2*>(F), p, reinterpret_cast<float2*>(ws), st));
    return forward_store_impl(box_geo(g), x, ws, p, prec, Y, at(ws, h), ws_bytes - h, st);
  }
  StepPlan sp;
  HICU_TRY(make_step_plan(g, p, prec, false, &sp));
  if (!ws || ws_bytes < sp.total) return HICU_ERR_WORKSPACE;
  {
    ProfScope ps("prep_weights", st, 0.0, 0.0, true);
    HICU_TRY(launch_prep_weights(0, prec, g, reinterpret_cast<const float2*>(F), p, sp.wf, at(ws, sp.off_Bf),
                                 at(ws, sp.off_Bflo), st));
  }
  fill_forward_args(g, x, sp, ws, reinterpret_cast<float*>(Y), reinterpret_cast<double*>(at(ws, sp.off_pf)));
  ConvPlan cf = sp.cf;
  cf.gy = group_col_blocks(cf, p);
  ProfScope ps(conv_tag(0, prec), st, 8.0 * g.n * (double)p * (double)g.s,
               8.0 * (double)region_points(g) * g.nc + 8.0 * (double)g.s * p);
  return launch_conv(cf, st);
}

size_t step_workspace(const Geo& g, int p, int prec) {
  if (g.kmasked) {
    const size_t inner = step_workspace(box_geo(g), p, prec);
    return inner ? kmask_head(g, p) + inner : 0;
  }
  StepPlan a, b;
  if (make_step_plan(g, p, prec, true, &a) != HICU_OK) return 0;
  if (make_step_plan(g, p, prec, false, &b) != HICU_OK) return 0;
  return std::max(a.total, b.total);
}


}  // namespace hicu
