// C ABI of the HICU hot-path library: argument validation, workspace
// planning and launch sequencing.  Every arithmetic step runs in the HIP
// kernels of conv.hip, gram.hip, eig.hip and ops.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "conv.h"
#include "eig.h"
#include "gram.h"
#include "ops.h"
#include "prof.h"

namespace hicu {

int32_t make_geo(const hicu_geom* gm, Geo* o) {
  if (!gm || !o) return HICU_ERR_ARG;
  const int nd = gm->ndim;
  if (nd < 1 || nd > 3 || gm->nchan < 1) return HICU_ERR_ARG;
  const int sh = 3 - nd;
  for (int a = 0; a < 3; ++a) {
    if (a < sh) {
      o->d[a] = 1;
      o->k[a] = 1;
      o->lo[a] = 0;
      o->hi[a] = 1;
    } else {
      o->d[a] = gm->dims[a - sh];
      o->k[a] = gm->kdims[a - sh];
      o->lo[a] = gm->lo[a - sh];
      o->hi[a] = gm->hi[a - sh];
    }
    if (o->d[a] < 1 || o->k[a] < 1 || o->k[a] > 64) return HICU_ERR_SHAPE;
    if (o->lo[a] < 0 || o->hi[a] > o->d[a] || o->hi[a] - o->lo[a] < o->k[a]) return HICU_ERR_SHAPE;
    o->m[a] = o->hi[a] - o->lo[a] - o->k[a] + 1;
  }
  o->nc = gm->nchan;
  const int64_t n = (int64_t)o->k[0] * o->k[1] * o->k[2] * o->nc;
  if (n > 16384) return HICU_ERR_SHAPE;
  o->n = (int)n;
  o->s = o->m[0] * o->m[1] * o->m[2];
  o->npts = o->d[0] * o->d[1] * o->d[2];
  if (o->npts > ((int64_t)1 << 40)) return HICU_ERR_SHAPE;
  return HICU_OK;
}

namespace {

constexpr size_t kAlign = 256;
inline size_t al(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

bool valid_prec(int p) { return p == P_F32 || p == P_BF16 || p == P_BF16X3; }
size_t esize(int prec) { return prec == P_F32 ? 4 : 2; }
int nparts(int prec) { return prec == P_BF16X3 ? 2 : 1; }

// Layout of the objective/gradient/line-search workspace.
struct StepPlan {
  WeightShape wf, wa;
  ConvPlan cf, ca;      // forward (also used for the line search), adjoint
  size_t off_Y, off_Bf, off_Bflo, off_Ba, off_Balo, off_pf, off_pa, off_pz, total;
  int64_t nf_blocks, na_blocks;
};

int32_t plan_forward(const Geo& g, int p, int prec, WeightShape* w, ConvPlan* c) {
  *w = weight_shape(prec, g.k, g.nc, g.nc, 2 * p);
  TileCfg t = default_tile(prec, g, 2 * p);
  int32_t s = plan_conv(prec, t, g.k, *w, w->nchunks, g.m, 2 * p, c);
  if (s == HICU_ERR_UNSUPPORTED && t.T0 > 1) {
    t.T0 = 1;
    t.T2 = 8;
    s = plan_conv(prec, t, g.k, *w, w->nchunks, g.m, 2 * p, c);
  }
  return s;
}

int32_t plan_adjoint(const Geo& g, int p, int prec, WeightShape* w, ConvPlan* c) {
  const int64_t oe[3] = {g.hi[0] - g.lo[0], g.hi[1] - g.lo[1], g.hi[2] - g.lo[2]};
  int32_t s = HICU_ERR_UNSUPPORTED;
  const TileCfg tiles[2] = {default_tile(prec, g, 2 * g.nc), TileCfg{1, 8, default_tile(prec, g, 2 * g.nc).WN}};
  for (const TileCfg& t : tiles) {
    for (int cc : {16, 8, 4}) {
      *w = weight_shape(prec, g.k, p, std::min(cc, std::max(1, p)), 2 * g.nc);
      s = plan_conv(prec, t, g.k, *w, w->nchunks, oe, 2 * g.nc, c);
      if (s != HICU_ERR_UNSUPPORTED) return s;
    }
  }
  return s;
}

int32_t make_step_plan(const Geo& g, int p, int prec, bool need_adj, StepPlan* sp) {
  HICU_TRY(plan_forward(g, p, prec, &sp->wf, &sp->cf));
  sp->nf_blocks = (int64_t)sp->cf.grid.x * sp->cf.grid.y;
  sp->na_blocks = 0;
  size_t off = 0;
  sp->off_Y = off;
  if (need_adj) off += al((size_t)g.s * p * sizeof(float2));
  sp->off_Bf = off;
  off += al(sp->wf.elems * esize(prec));
  sp->off_Bflo = off;
  if (prec == P_BF16X3) off += al(sp->wf.elems * esize(prec));
  sp->off_Ba = sp->off_Balo = off;
  if (need_adj) {
    HICU_TRY(plan_adjoint(g, p, prec, &sp->wa, &sp->ca));
    sp->na_blocks = (int64_t)sp->ca.grid.x * sp->ca.grid.y;
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
  sp->total = off;
  return HICU_OK;
}

// Profiler tag of a contraction: kind (0 forward, 1 adjoint, 2 line search) x precision.
const char* conv_tag(int kind, int prec) {
  static const char* tags[3][3] = {{"conv_fwd_fp32", "conv_fwd_bf16", "conv_fwd_bf16x3"},
                                   {"conv_adj_fp32", "conv_adj_bf16", "conv_adj_bf16x3"},
                                   {"conv_els_fp32", "conv_els_bf16", "conv_els_bf16x3"}};
  return tags[kind][prec];
}

inline char* at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

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
  a.ch0 = 0;
  for (int i = 0; i < 3; ++i) {
    a.vlo[i] = 0;
    a.vhi[i] = g.d[i];
    a.org[i] = g.lo[i];
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
}

// Objective, gradient; shared by the public entry and the solver loop.
int32_t objective_grad_impl(const Geo& g, const void* x, const uint8_t* mask, const void* F, int p, int prec,
                            double* J, void* gout, double* gn2, void* ws, size_t ws_bytes, hipStream_t st) {
  StepPlan sp;
  HICU_TRY(make_step_plan(g, p, prec, gout != nullptr, &sp));
  if (!ws || ws_bytes < sp.total) return HICU_ERR_WORKSPACE;
  const float2* Fc = reinterpret_cast<const float2*>(F);
  const double flops = 8.0 * g.n * (double)p * (double)g.s;
  const double nS = (double)region_points(g);
  {
    ProfScope ps("prep_weights", st);
    HICU_TRY(launch_prep_weights(0, prec, g, Fc, p, sp.wf, at(ws, sp.off_Bf), at(ws, sp.off_Bflo), st));
  }
  float2* Y = reinterpret_cast<float2*>(at(ws, sp.off_Y));
  double* pf = reinterpret_cast<double*>(at(ws, sp.off_pf));
  fill_forward_args(g, x, sp, ws, gout ? reinterpret_cast<float*>(Y) : nullptr, pf);
  {
    ProfScope ps(conv_tag(0, prec), st, flops, 8.0 * (nS * g.nc + (gout ? (double)g.s * p : 0.0)));
    HICU_TRY(launch_conv(sp.cf, st));
  }
  if (J) {
    ProfScope ps("reduce", st);
    HICU_TRY(launch_reduce(pf, sp.nf_blocks, J, st));
  }
  if (!gout) return HICU_OK;
  if (!full_region(g)) {
    ProfScope ps("zero", st);
    HICU_TRY(launch_zero(gout, (size_t)g.npts * g.nc * sizeof(float2), st));
  }
  {
    ProfScope ps("prep_weights", st);
    HICU_TRY(launch_prep_weights(1, prec, g, Fc, p, sp.wa, at(ws, sp.off_Ba), at(ws, sp.off_Balo), st));
  }
  ConvArgs& a = sp.ca.a;
  a.in = Y;
  a.is[0] = g.m[1] * g.m[2] * p;
  a.is[1] = g.m[2] * p;
  a.is[2] = p;
  a.cin = p;
  a.ch0 = 0;
  for (int i = 0; i < 3; ++i) {
    a.vlo[i] = 0;
    a.vhi[i] = g.m[i];
    a.org[i] = -(int64_t)(g.k[i] - 1);
  }
  a.B = at(ws, sp.off_Ba);
  a.Blo = at(ws, sp.off_Balo);
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
  double* pa = reinterpret_cast<double*>(at(ws, sp.off_pa));
  a.partial = pa;
  {
    ProfScope ps(conv_tag(1, prec), st, flops, 8.0 * ((double)g.s * p + nS * g.nc) + nS);
    HICU_TRY(launch_conv(sp.ca, st));
  }
  if (gn2) {
    ProfScope ps("reduce", st);
    HICU_TRY(launch_reduce(pa, sp.na_blocks, gn2, st));
  }
  return HICU_OK;
}

int32_t line_search_impl(const Geo& g, const void* gv, const double* gn2, const void* F, int p, int prec,
                         double* eta, void* ws, size_t ws_bytes, hipStream_t st) {
  StepPlan sp;
  HICU_TRY(make_step_plan(g, p, prec, false, &sp));
  // The line-search layout is a prefix-compatible subset of the gradient
  // layout only when no Y is stored, so use its own offsets.
  if (!ws || ws_bytes < sp.total) return HICU_ERR_WORKSPACE;
  {
    ProfScope ps("prep_weights", st);
    HICU_TRY(launch_prep_weights(0, prec, g, reinterpret_cast<const float2*>(F), p, sp.wf, at(ws, sp.off_Bf),
                                 at(ws, sp.off_Bflo), st));
  }
  double* pz = reinterpret_cast<double*>(at(ws, sp.off_pz));
  fill_forward_args(g, gv, sp, ws, nullptr, pz);
  {
    ProfScope ps(conv_tag(2, prec), st, 8.0 * g.n * (double)p * (double)g.s, 8.0 * (double)region_points(g) * g.nc);
    HICU_TRY(launch_conv(sp.cf, st));
  }
  {
    ProfScope ps("eta", st);
    HICU_TRY(launch_eta(pz, sp.nf_blocks, gn2, eta, st));
  }
  return HICU_OK;
}

size_t step_workspace(const Geo& g, int p, int prec) {
  StepPlan a, b;
  if (make_step_plan(g, p, prec, true, &a) != HICU_OK) return 0;
  if (make_step_plan(g, p, prec, false, &b) != HICU_OK) return 0;
  return std::max(a.total, b.total);
}

}  // namespace
}  // namespace hicu

using namespace hicu;

extern "C" {

int32_t hicu_version(void) { return 100; }

const char* hicu_status_string(int32_t s) {
  switch (s) {
    case HICU_OK: return "ok";
    case HICU_CONVERGED: return "converged (zero gradient)";
    case HICU_ERR_ARG: return "invalid argument";
    case HICU_ERR_SHAPE: return "invalid geometry";
    case HICU_ERR_RANK: return "rank or filter count out of range";
    case HICU_ERR_NONFINITE: return "non-finite value";
    case HICU_ERR_HIP: return "HIP runtime error";
    case HICU_ERR_WORKSPACE: return "workspace missing or too small";
    case HICU_ERR_UNSUPPORTED: return "unsupported configuration";
    case HICU_ERR_NOCONV: return "eigensolver did not converge";
    default: return "unknown status";
  }
}

int64_t hicu_num_taps(const hicu_geom* gm) {
  Geo g;
  const int32_t s = make_geo(gm, &g);
  return s < 0 ? s : g.n;
}

int64_t hicu_num_outputs(const hicu_geom* gm) {
  Geo g;
  const int32_t s = make_geo(gm, &g);
  return s < 0 ? s : g.s;
}

size_t hicu_gram_workspace_bytes(const hicu_geom* gm) {
  Geo g;
  if (make_geo(gm, &g) != HICU_OK) return 0;
  return gram_workspace(g);
}

int32_t hicu_gram(const hicu_geom* gm, const void* x, void* G, void* ws, size_t ws_bytes, void* stream) {
  Geo g;
  HICU_TRY(make_geo(gm, &g));
  if (!x || !G) return HICU_ERR_ARG;
  ProfScope ps("gram", (hipStream_t)stream, 8.0 * (double)g.s * g.n * g.n, 8.0 * region_points(g) * g.nc);
  return launch_gram(g, x, G, ws, ws_bytes, (hipStream_t)stream);
}

size_t hicu_nullspace_workspace_bytes(int32_t n) { return n < 1 ? 0 : eig_workspace(n); }

int32_t hicu_nullspace(int32_t n, int32_t rank, const void* G, const void* V0, void* Q, double* evals, void* V,
                       int32_t* sweeps, void* ws, size_t ws_bytes, void* stream) {
  if (n < 1 || n > 16384) return HICU_ERR_ARG;
  if (rank < 0 || rank >= n) return HICU_ERR_RANK;
  if (!G || (!Q && !V && !evals)) return HICU_ERR_ARG;
  ProfScope ps("eig", (hipStream_t)stream);
  return run_eig(n, rank, G, V0, Q, evals, V, sweeps, ws, ws_bytes, (hipStream_t)stream, false);
}

int32_t hicu_jl_compress(int32_t n, int32_t nq, int32_t p, const void* Q, uint64_t seed, uint32_t outer,
                         uint32_t inner, uint32_t sid, void* F, double* P, void* stream) {
  if (n < 1 || nq < 1 || p < 1 || !Q || !F) return HICU_ERR_ARG;
  ProfScope ps("jl", (hipStream_t)stream);
  return launch_jl(reinterpret_cast<const float2*>(Q), n, nq, p, seed, outer, inner, sid,
                   reinterpret_cast<float2*>(F), P, (hipStream_t)stream);
}

size_t hicu_workspace_bytes(const hicu_geom* gm, int32_t p, int32_t prec) {
  Geo g;
  if (make_geo(gm, &g) != HICU_OK || p < 1 || !valid_prec(prec)) return 0;
  return step_workspace(g, p, prec);
}

int32_t hicu_objective_grad(const hicu_geom* gm, const void* x, const uint8_t* mask, const void* F, int32_t p,
                            int32_t prec, double* J, void* gout, double* gn2, void* ws, size_t ws_bytes,
                            void* stream) {
  Geo g;
  HICU_TRY(make_geo(gm, &g));
  if (!x || !F || !valid_prec(prec)) return HICU_ERR_ARG;
  if (p < 1 || p > 1 << 20) return HICU_ERR_RANK;
  if (gn2 && !gout) return HICU_ERR_ARG;
  return objective_grad_impl(g, x, mask, F, p, prec, J, gout, gn2, ws, ws_bytes, (hipStream_t)stream);
}

int32_t hicu_line_search(const hicu_geom* gm, const void* gv, const double* gn2, const void* F, int32_t p,
                         int32_t prec, double* eta, void* ws, size_t ws_bytes, void* stream) {
  Geo g;
  HICU_TRY(make_geo(gm, &g));
  if (!gv || !gn2 || !F || !eta || !valid_prec(prec)) return HICU_ERR_ARG;
  if (p < 1 || p > 1 << 20) return HICU_ERR_RANK;
  return line_search_impl(g, gv, gn2, F, p, prec, eta, ws, ws_bytes, (hipStream_t)stream);
}

int32_t hicu_update(const hicu_geom* gm, void* x, const void* gv, const double* eta, void* stream) {
  Geo g;
  HICU_TRY(make_geo(gm, &g));
  if (!x || !gv || !eta) return HICU_ERR_ARG;
  ProfScope ps("update", (hipStream_t)stream, 0.0, 24.0 * (double)g.npts * g.nc);
  return launch_update(reinterpret_cast<float2*>(x), reinterpret_cast<const float2*>(gv), eta,
                       g.npts * g.nc, (hipStream_t)stream);
}

int32_t hicu_solve(const hicu_geom* gm, const void* x0, const uint8_t* mask, const hicu_params* prm, void* xout,
                   hicu_trace* trace, void* stream) {
  Geo full;
  HICU_TRY(make_geo(gm, &full));
  if (!x0 || !xout || !prm || !prm->steps) return HICU_ERR_ARG;
  if (!valid_prec(prm->prec) || prm->n_outer < 0 || prm->start_outer < 0 || prm->refine_steps < 0)
    return HICU_ERR_ARG;
  const int n = full.n, r = prm->rank;
  if (r < 0 || r >= n) return HICU_ERR_RANK;
  const int nq = n - r;
  if (prm->p < 0) return HICU_ERR_RANK;
  const int pf = prm->p == 0 ? nq : prm->p;
  hipStream_t st = (hipStream_t)stream;
  // Per-iteration geometries (validated up front: nothing runs on bad input).
  std::vector<Geo> geos(prm->n_outer);
  int64_t total_steps = 0;
  for (int i = 0; i < prm->n_outer; ++i) {
    hicu_geom gi = *gm;
    if (prm->regions) {
      for (int a = 0; a < gm->ndim; ++a) {
        gi.lo[a] = prm->regions[i * 6 + a];
        gi.hi[a] = prm->regions[i * 6 + 3 + a];
      }
    }
    HICU_TRY(make_geo(&gi, &geos[i]));
    if (prm->steps[i] < 0) return HICU_ERR_ARG;
    if (i >= prm->start_outer) total_steps += prm->steps[i];
  }
  size_t ws_step = 0;
  for (int i = prm->start_outer; i < prm->n_outer; ++i) {
    ws_step = std::max(ws_step, step_workspace(geos[i], pf, prm->prec));
    ws_step = std::max(ws_step, step_workspace(geos[i], pf, P_F32));
    if (ws_step == 0) return HICU_ERR_UNSUPPORTED;
  }
  size_t ws_gram = 0;
  for (int i = prm->start_outer; i < prm->n_outer; ++i) ws_gram = std::max(ws_gram, gram_workspace(geos[i]));
  const size_t N = (size_t)full.npts * full.nc;
  size_t off = 0;
  const size_t o_g = off; off += al(N * sizeof(float2));
  const size_t o_G = off; off += al((size_t)n * n * sizeof(double2));
  const size_t o_V0 = off; off += al((size_t)n * n * sizeof(double2));
  const size_t o_V1 = off; off += al((size_t)n * n * sizeof(double2));
  const size_t o_Q = off; off += al((size_t)n * nq * sizeof(float2));
  const size_t o_F = off; off += al((size_t)n * pf * sizeof(float2));
  const size_t o_sc = off; off += al((size_t)std::max<int64_t>(1, total_steps) * 3 * sizeof(double));
  const size_t o_eig = off; off += al(eig_workspace(n));
  const size_t o_gram = off; off += al(ws_gram);
  const size_t o_step = off; off += al(ws_step);
  void* ws = nullptr;
  HICU_HIP_TRY(hipMalloc(&ws, off));
  struct Free {
    void* p;
    ~Free() { if (p) (void)hipFree(p); }
  } guard{ws};
  float2* x = reinterpret_cast<float2*>(xout);
  float2* g = reinterpret_cast<float2*>(at(ws, o_g));
  double* sc = reinterpret_cast<double*>(at(ws, o_sc));
  if (xout != x0) HICU_HIP_TRY(hipMemcpyAsync(xout, x0, N * sizeof(float2), hipMemcpyDeviceToDevice, st));
  std::vector<int32_t> sweeps_of(prm->n_outer, 0);
  void* Vprev = at(ws, o_V0);
  void* Vcur = at(ws, o_V1);
  bool have_prev = false;
  int32_t status = HICU_OK;
  int64_t step = 0;
  std::vector<int32_t> prec_of(std::max<int64_t>(1, total_steps));
  std::vector<int32_t> outer_of(prec_of.size()), inner_of(prec_of.size());
  for (int i = prm->start_outer; i < prm->n_outer; ++i) {
    const Geo& gi = geos[i];
    {
      ProfScope ps("gram", st, 8.0 * (double)gi.s * n * n, 8.0 * region_points(gi) * gi.nc);
      HICU_TRY(launch_gram(gi, x, at(ws, o_G), at(ws, o_gram), ws_gram, st));
    }
    int32_t sw = 0;
    int32_t es;
    {
      ProfScope ps("eig", st);
      es = run_eig(n, r, at(ws, o_G), (prm->warm_start && have_prev) ? Vprev : nullptr, at(ws, o_Q), nullptr, Vcur,
                   &sw, at(ws, o_eig), eig_workspace(n), st,
                   prm->p == 0);
    }
    if (es < 0 && es != HICU_ERR_NOCONV) return es;
    if (es == HICU_ERR_NOCONV) status = HICU_ERR_NOCONV;
    sweeps_of[i] = sw;
    std::swap(Vprev, Vcur);
    have_prev = true;
    for (int j = 0; j < prm->steps[i]; ++j, ++step) {
      const int prec = (step >= total_steps - prm->refine_steps) ? P_F32 : prm->prec;
      prec_of[step] = prec;
      outer_of[step] = i;
      inner_of[step] = j;
      const void* F = at(ws, o_Q);
      if (prm->p > 0) {
        ProfScope ps("jl", st);
        HICU_TRY(launch_jl(reinterpret_cast<const float2*>(at(ws, o_Q)), n, nq, pf, prm->seed, (uint32_t)i,
                           (uint32_t)j, 0u, reinterpret_cast<float2*>(at(ws, o_F)), nullptr, st));
        F = at(ws, o_F);
      }
      double* Jd = sc + 3 * step;
      HICU_TRY(objective_grad_impl(gi, x, mask, F, pf, prec, Jd, g, Jd + 1, at(ws, o_step), ws_step, st));
      HICU_TRY(line_search_impl(gi, g, Jd + 1, F, pf, prec, Jd + 2, at(ws, o_step), ws_step, st));
      ProfScope ps("update", st, 0.0, 24.0 * (double)N);
      HICU_TRY(launch_update(x, g, Jd + 2, (int64_t)N, st));
    }
  }
  std::vector<double> hs((size_t)std::max<int64_t>(1, total_steps) * 3);
  if (total_steps > 0)
    HICU_HIP_TRY(hipMemcpyAsync(hs.data(), sc, (size_t)total_steps * 3 * sizeof(double), hipMemcpyDeviceToHost, st));
  HICU_HIP_TRY(hipStreamSynchronize(st));
  for (int64_t s = 0; s < total_steps; ++s) {
    if (!std::isfinite(hs[3 * s]) || !std::isfinite(hs[3 * s + 1])) status = HICU_ERR_NONFINITE;
    if (trace) {
      trace[s].outer = outer_of[s];
      trace[s].inner = inner_of[s];
      trace[s].prec = prec_of[s];
      trace[s].sweeps = sweeps_of[outer_of[s]];
      trace[s].J = hs[3 * s];
      trace[s].gnorm2 = hs[3 * s + 1];
      trace[s].eta = hs[3 * s + 2];
    }
  }
  return status;
}

}  // extern "C"
