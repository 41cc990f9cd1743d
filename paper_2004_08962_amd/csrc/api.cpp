// C ABI of the HICU hot-path library: argument validation, workspace
// planning and launch sequencing.  Every arithmetic step runs in the HIP
// kernels of conv.hip, gram.hip, eig.hip, rsvd.hip and ops.hip.
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
#include "rsvd.h"
#include "step.h"

namespace hicu {

int32_t make_geo(const hicu_geom* gm, Geo* o) {
  if (!gm || !o) return HICU_ERR_ARG;
  const int nd = gm->ndim;
  if (nd < 1 || nd > 3 || gm->nchan < 1) return HICU_ERR_ARG;
  const int sh = 3 - nd;
  if (gm->wrap < 0 || gm->wrap >= (1 << nd)) return HICU_ERR_ARG;
  for (int a = 0; a < 3; ++a) {
    if (a < sh) {
      o->d[a] = 1;
      o->k[a] = 1;
      o->lo[a] = 0;
      o->hi[a] = 1;
      o->wrap[a] = 0;
    } else {
      o->d[a] = gm->dims[a - sh];
      o->k[a] = gm->kdims[a - sh];
      o->lo[a] = gm->lo[a - sh];
      o->hi[a] = gm->hi[a - sh];
      o->wrap[a] = (gm->wrap >> (a - sh)) & 1;
    }
    if (o->d[a] < 1 || o->k[a] < 1 || o->k[a] > 64) return HICU_ERR_SHAPE;
    if (o->lo[a] < 0 || o->hi[a] > o->d[a] || o->hi[a] - o->lo[a] < o->k[a]) return HICU_ERR_SHAPE;
    if (o->wrap[a] && (o->lo[a] != 0 || o->hi[a] != o->d[a])) return HICU_ERR_SHAPE;
    o->m[a] = o->wrap[a] ? o->d[a] : o->hi[a] - o->lo[a] - o->k[a] + 1;
  }
  o->nc = gm->nchan;
  const int64_t box = (int64_t)o->k[0] * o->k[1] * o->k[2];
  const int64_t n = box * o->nc;
  if (n > 16384) return HICU_ERR_SHAPE;
  o->n = (int)n;
  o->nbox = (int)n;
  o->kmasked = 0;
  for (int w = 0; w < 8; ++w) o->kbits[w] = 0;
  if (gm->kmask) {
    if (box > 512) return HICU_ERR_UNSUPPORTED;
    int taps = 0;
    for (int64_t f = 0; f < box; ++f)
      if (gm->kmask[f]) {
        o->kbits[f >> 6] |= 1ull << (f & 63);
        ++taps;
      }
    if (taps == 0) return HICU_ERR_SHAPE;
    if (taps < box) {
      o->kmasked = 1;
      o->n = taps * o->nc;
    }
  }
  o->s = o->m[0] * o->m[1] * o->m[2];
  o->npts = o->d[0] * o->d[1] * o->d[2];
  if (o->npts > ((int64_t)1 << 40)) return HICU_ERR_SHAPE;
  return HICU_OK;
}

Geo box_geo(const Geo& g) {
  Geo b = g;
  b.kmasked = 0;
  b.n = g.nbox;
  return b;
}

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
  ProfScope ps("gram", (hipStream_t)stream, 4.0 * (double)g.s * g.n * g.n, 8.0 * region_points(g) * g.nc);
  return launch_gram(g, x, G, ws, ws_bytes, (hipStream_t)stream);
}

int32_t hicu_set_gram_route(int32_t route) {
  if (route != 0 && route != 1) return HICU_ERR_ARG;
  set_gram_route(route);
  return HICU_OK;
}

size_t hicu_nullspace_workspace_bytes(int32_t n) { return n < 1 ? 0 : eig_workspace(n); }

int32_t hicu_nullspace(int32_t n, int32_t rank, const void* G, const void* V0, void* Q, double* evals, void* V,
                       int32_t* sweeps, void* ws, size_t ws_bytes, void* stream) {
  if (n < 1 || n > 16384) return HICU_ERR_ARG;
  if (rank < 0 || rank >= n) return HICU_ERR_RANK;
  if (!G || (!Q && !V && !evals)) return HICU_ERR_ARG;
  ProfScope ps("eig", (hipStream_t)stream);
  const int32_t s = run_eig(n, rank, G, V0, Q, evals, V, sweeps, ws, ws_bytes, (hipStream_t)stream, false);
  // wait for the queued work unless the call was rejected before any launch
  if (s == HICU_OK || s == HICU_ERR_NOCONV || s == HICU_ERR_NONFINITE) {
    HostWait w;
    HICU_HIP_TRY(w.stream((hipStream_t)stream));
  }
  return s;
}

size_t hicu_nullspace_rsvd_workspace_bytes(const hicu_geom* gm, int32_t rank, int32_t ell) {
  Geo g;
  if (make_geo(gm, &g) != HICU_OK || rank < 0 || rank >= g.n || g.n > kRsvdMaxN) return 0;
  if (rank == 0) return 256;
  const int l = ell == 0 ? default_sketch(rank, g.n) : ell;
  if (l < rank || l > g.n) return 0;
  return rsvd_workspace(g, rank, l);
}

int32_t hicu_nullspace_rsvd(const hicu_geom* gm, const void* x, int32_t rank, int32_t ell, uint64_t seed,
                            uint32_t outer, uint32_t sid, void* Q, double* sv, int32_t* sweeps, void* ws,
                            size_t ws_bytes, void* stream) {
  Geo g;
  HICU_TRY(make_geo(gm, &g));
  if (!x || !Q) return HICU_ERR_ARG;
  if (rank < 0 || rank >= g.n) return HICU_ERR_RANK;
  if (g.n > kRsvdMaxN) return HICU_ERR_UNSUPPORTED;
  const int l = ell == 0 ? default_sketch(rank, g.n) : ell;
  if (rank > 0 && (l < rank || l > g.n)) return HICU_ERR_ARG;
  ProfScope ps("rsvd", (hipStream_t)stream);
  const int32_t s = run_rsvd(g, x, rank, l, seed, outer, sid, reinterpret_cast<float2*>(Q), sv, sweeps, ws,
                             ws_bytes, (hipStream_t)stream, true);
  // wait for the queued work unless the call was rejected before any launch
  if (s == HICU_OK || s == HICU_ERR_NOCONV || s == HICU_ERR_NONFINITE) {
    HostWait w;
    HICU_HIP_TRY(w.stream((hipStream_t)stream));
  }
  return s;
}

int32_t hicu_sketch(int32_t n, int32_t ell, uint64_t seed, uint32_t outer, uint32_t sid, void* Om, void* stream) {
  if (n < 1 || ell < 1 || !Om) return HICU_ERR_ARG;
  return launch_sketch(n, ell, seed, outer, sid, reinterpret_cast<float2*>(Om), (hipStream_t)stream);
}

int32_t hicu_jl_compress(int32_t n, int32_t nq, int32_t p, const void* Q, uint64_t seed, uint32_t outer,
                         uint32_t inner, uint32_t sid, void* F, double* P, void* stream) {
  if (n < 1 || nq < 1 || p < 1 || !Q || !F) return HICU_ERR_ARG;
  ProfScope ps("jl", (hipStream_t)stream);
  return launch_jl(reinterpret_cast<const float2*>(Q), n, nq, p, seed, outer, inner, sid,
                   reinterpret_cast<float2*>(F), P, (hipStream_t)stream);
}

int32_t hicu_set_filter_group_budget(size_t bytes) {
  set_y_budget(bytes);
  return HICU_OK;
}

int32_t hicu_filter_group(const hicu_geom* gm, int32_t p, int32_t prec, int32_t* filters, int32_t* compact) {
  if (!filters) return HICU_ERR_ARG;
  Geo g;
  HICU_TRY(make_geo(gm, &g));
  if (p < 1 || !valid_prec(prec)) return HICU_ERR_ARG;
  StepPlan sp;
  HICU_TRY(make_step_plan(g, p, prec, true, &sp));
  *filters = sp.pc;
  if (compact) *compact = sp.ybw > 0;
  return HICU_OK;
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

int32_t hicu_time_average_init(const hicu_geom* gm, int32_t axis, const void* x0, const uint8_t* mask, void* xout,
                               void* stream) {
  Geo g;
  HICU_TRY(make_geo(gm, &g));
  if (!x0 || !mask || !xout || axis < 0 || axis >= gm->ndim) return HICU_ERR_ARG;
  ProfScope ps("time_average", (hipStream_t)stream, 0.0, 16.0 * (double)g.npts * g.nc + (double)g.npts);
  return launch_time_average(reinterpret_cast<const float2*>(x0), mask, reinterpret_cast<float2*>(xout), g.d,
                             axis + (3 - gm->ndim), g.nc, (hipStream_t)stream);
}

int32_t hicu_update(const hicu_geom* gm, void* x, const void* gv, const double* eta, void* stream) {
  Geo g;
  HICU_TRY(make_geo(gm, &g));
  if (!x || !gv || !eta) return HICU_ERR_ARG;
  ProfScope ps("update", (hipStream_t)stream, 0.0, 24.0 * (double)g.npts * g.nc, true);
  return launch_update(reinterpret_cast<float2*>(x), reinterpret_cast<const float2*>(gv), eta,
                       g.npts * g.nc, (hipStream_t)stream);
}

}  // extern "C"

namespace hicu {
namespace {

// Validated per-iteration geometries and the workspace layout of hicu_solve.
struct SolvePlan {
  std::vector<Geo> geos;
  int64_t total_steps = 0;
  int n = 0, nq = 0, pf = 0;
  int ell = 0;
  size_t ws_step = 0, ws_gram = 0, ws_rsvd = 0;
  size_t o_g, o_G, o_V0, o_V1, o_Q, o_F, o_sc, o_cnt, o_eig, o_gram, o_rsvd, o_step, total;
};

int32_t make_solve_plan(const hicu_geom* gm, const hicu_params* prm, SolvePlan* sp) {
  Geo full;
  HICU_TRY(make_geo(gm, &full));
  if (!prm || !prm->steps) return HICU_ERR_ARG;
  if (!valid_prec(prm->prec) || prm->n_outer < 0 || prm->start_outer < 0 || prm->refine_steps < 0)
    return HICU_ERR_ARG;
  if (prm->refine_prec != P_F32 && prm->refine_prec != P_BF16X3) return HICU_ERR_ARG;
  const int n = full.n, r = prm->rank;
  if (r < 0 || r >= n) return HICU_ERR_RANK;
  if (prm->p < 0) return HICU_ERR_RANK;
  if (prm->route != 0 && prm->route != 1) return HICU_ERR_ARG;
  const bool rsvd = prm->route == 1;
  if (rsvd) {
    if (n > kRsvdMaxN) return HICU_ERR_UNSUPPORTED;
    sp->ell = prm->sketch == 0 ? default_sketch(r, n) : prm->sketch;
    if (r > 0 && (sp->ell < r || sp->ell > n)) return HICU_ERR_ARG;
  }
  sp->n = n;
  sp->nq = n - r;
  sp->pf = prm->p == 0 ? sp->nq : prm->p;
  sp->geos.assign(prm->n_outer, Geo{});
  sp->total_steps = 0;
  for (int i = 0; i < prm->n_outer; ++i) {
    hicu_geom gi = *gm;
    if (prm->regions) {
      for (int a = 0; a < gm->ndim; ++a) {
        gi.lo[a] = prm->regions[i * 6 + a];
        gi.hi[a] = prm->regions[i * 6 + 3 + a];
      }
    }
    HICU_TRY(make_geo(&gi, &sp->geos[i]));
    if (prm->steps[i] < 0) return HICU_ERR_ARG;
    if (i >= prm->start_outer) sp->total_steps += prm->steps[i];
  }
  sp->ws_step = sp->ws_gram = sp->ws_rsvd = 0;
  for (int i = prm->start_outer; i < prm->n_outer; ++i) {
    const size_t a = step_workspace(sp->geos[i], sp->pf, prm->prec),
                 b = step_workspace(sp->geos[i], sp->pf, prm->refine_prec);
    if (a == 0 || b == 0) return HICU_ERR_UNSUPPORTED;
    sp->ws_step = std::max(sp->ws_step, std::max(a, b));
    if (rsvd) {
      const size_t w = r == 0 ? 256 : rsvd_workspace(sp->geos[i], r, sp->ell);
      if (w == 0) return HICU_ERR_UNSUPPORTED;
      sp->ws_rsvd = std::max(sp->ws_rsvd, w);
    } else {
      sp->ws_gram = std::max(sp->ws_gram, gram_workspace(sp->geos[i]));
    }
  }
  // The Gram route keeps G, two eigenvector sets (warm start) and the
  // eigensolver's workspace; the rSVD route only its own workspace.
  const size_t N = (size_t)full.npts * full.nc;
  const size_t nn = rsvd ? 0 : (size_t)n * n * sizeof(double2);
  size_t off = 0;
  sp->o_g = off; off += al(N * sizeof(float2));
  sp->o_G = off; off += al(nn);
  sp->o_V0 = off; off += al(nn);
  sp->o_V1 = off; off += al(nn);
  sp->o_Q = off; off += al((size_t)n * sp->nq * sizeof(float2));
  sp->o_F = off; off += al((size_t)n * sp->pf * sizeof(float2));
  sp->o_sc = off; off += al((size_t)std::max<int64_t>(1, sp->total_steps) * 3 * sizeof(double));
  sp->o_cnt = off; off += al(sizeof(unsigned long long));
  sp->o_eig = off; off += al(rsvd ? 0 : eig_workspace(n));
  sp->o_gram = off; off += al(sp->ws_gram);
  sp->o_rsvd = off; off += al(sp->ws_rsvd);
  sp->o_step = off; off += al(sp->ws_step);
  sp->total = off;
  return HICU_OK;
}

}  // namespace
}  // namespace hicu

extern "C" {

size_t hicu_solve_workspace_bytes(const hicu_geom* gm, const hicu_params* prm) {
  SolvePlan sp;
  return make_solve_plan(gm, prm, &sp) == HICU_OK ? sp.total : 0;
}

int32_t hicu_solve(const hicu_geom* gm, const void* x0, const uint8_t* mask, const hicu_params* prm, void* xout,
                   hicu_trace* trace, void* ws, size_t ws_bytes, void* stream) {
  SolvePlan pl;
  HICU_TRY(make_solve_plan(gm, prm, &pl));
  if (!x0 || !xout) return HICU_ERR_ARG;
  if (!ws || ws_bytes < pl.total) return HICU_ERR_WORKSPACE;
  Geo full;
  HICU_TRY(make_geo(gm, &full));
  const int n = pl.n, r = prm->rank, nq = pl.nq, pf = pl.pf;
  const int64_t total_steps = pl.total_steps;
  hipStream_t st = (hipStream_t)stream;
  const size_t N = (size_t)full.npts * full.nc;
  float2* x = reinterpret_cast<float2*>(xout);
  float2* g = reinterpret_cast<float2*>(at(ws, pl.o_g));
  double* sc = reinterpret_cast<double*>(at(ws, pl.o_sc));
  HostWait wait;
  // A non-finite input is rejected before anything is written.
  {
    unsigned long long bad = 0;
    auto* cnt = reinterpret_cast<unsigned long long*>(at(ws, pl.o_cnt));
    HICU_TRY(launch_count_nonfinite(reinterpret_cast<const float*>(x0), 2 * (int64_t)N, cnt, st));
    HICU_HIP_TRY(hipMemcpyAsync(&bad, cnt, sizeof(bad), hipMemcpyDeviceToHost, st));
    HICU_HIP_TRY(hipStreamSynchronize(st));
    if (bad) return HICU_ERR_NONFINITE;
  }
  if (xout != x0) HICU_HIP_TRY(hipMemcpyAsync(xout, x0, N * sizeof(float2), hipMemcpyDeviceToDevice, st));
  void* Vprev = at(ws, pl.o_V0);
  void* Vcur = at(ws, pl.o_V1);
  bool have_prev = false;
  int32_t status = HICU_OK;
  int64_t step = 0;
  std::vector<double> hs(3 * (size_t)std::max<int64_t>(1, total_steps));
  for (int i = prm->start_outer; i < prm->n_outer && status != HICU_ERR_NONFINITE; ++i) {
    const Geo& gi = pl.geos[i];
    int32_t sw = 0;
    int32_t es;
    if (prm->route == 1) {
      ProfScope ps("rsvd", st);
      es = run_rsvd(gi, x, r, pl.ell, prm->seed, (uint32_t)i, 0u, reinterpret_cast<float2*>(at(ws, pl.o_Q)),
                    nullptr, &sw, at(ws, pl.o_rsvd), pl.ws_rsvd, st, prm->p > 0);
    } else {
      {
        ProfScope ps("gram", st, 4.0 * (double)gi.s * n * n, 8.0 * region_points(gi) * gi.nc);
        HICU_TRY(launch_gram(gi, x, at(ws, pl.o_G), at(ws, pl.o_gram), pl.ws_gram, st));
      }
      ProfScope ps("eig", st);
      es = run_eig(n, r, at(ws, pl.o_G), (prm->warm_start && have_prev) ? Vprev : nullptr, at(ws, pl.o_Q), nullptr,
                   Vcur, &sw, at(ws, pl.o_eig), eig_workspace(n), st, prm->p == 0);
      std::swap(Vprev, Vcur);
      have_prev = true;
    }
    if (es < 0 && es != HICU_ERR_NOCONV) return es;
    if (es == HICU_ERR_NOCONV) status = HICU_ERR_NOCONV;
    const int64_t step0 = step;
    int prepped_prec = -1;  // precision whose weights of this iteration's F are in the workspace
    for (int j = 0; j < prm->steps[i]; ++j, ++step) {
      const int prec = (step >= total_steps - prm->refine_steps) ? prm->refine_prec : prm->prec;
      if (trace) {
        trace[step].outer = i;
        trace[step].inner = j;
        trace[step].prec = prec;
        trace[step].sweeps = sw;
      }
      const void* F = at(ws, pl.o_Q);
      if (prm->p > 0) {
        ProfScope ps("jl", st);
        HICU_TRY(launch_jl(reinterpret_cast<const float2*>(at(ws, pl.o_Q)), n, nq, pf, prm->seed, (uint32_t)i,
                           (uint32_t)j, 0u, reinterpret_cast<float2*>(at(ws, pl.o_F)), nullptr, st));
        F = at(ws, pl.o_F);
        prepped_prec = -1;  // a new F every step
      }
      // Without JL the filters are fixed for the whole outer iteration, so
      // their weight layouts are built once (again when the precision switches).
      const int prep = prec == prepped_prec ? 0 : kPrepAll;
      prepped_prec = prec;
      double* Jd = sc + 3 * step;
      HICU_TRY(objective_grad_impl(gi, x, mask, F, pf, prec, Jd, g, Jd + 1, at(ws, pl.o_step), pl.ws_step, st, prep));
      HICU_TRY(line_search_impl(gi, g, Jd + 1, F, pf, prec, Jd + 2, at(ws, pl.o_step), pl.ws_step, st, true));
      ProfScope ps("update", st, 0.0, 24.0 * (double)N, true);
      HICU_TRY(launch_update(x, g, Jd + 2, (int64_t)N, st));
    }
    // The step scalars of this iteration: a non-finite J or gradient stops the
    // run.  The line search turns any non-finite scalar into a zero step and
    // the update skips zero steps, so x stays at its last finite iterate.
    const int64_t cnt = step - step0;
    if (cnt > 0) {
      HICU_HIP_TRY(hipMemcpyAsync(hs.data() + 3 * step0, sc + 3 * step0, (size_t)cnt * 3 * sizeof(double),
                                  hipMemcpyDeviceToHost, st));
      HICU_HIP_TRY(wait.stream(st));
    }
    for (int64_t s = step0; s < step; ++s) {
      if (!std::isfinite(hs[3 * s]) || !std::isfinite(hs[3 * s + 1]) || !std::isfinite(hs[3 * s + 2]))
        status = HICU_ERR_NONFINITE;
      if (trace) {
        trace[s].J = hs[3 * s];
        trace[s].gnorm2 = hs[3 * s + 1];
        trace[s].eta = hs[3 * s + 2];
      }
    }
  }
  // Steps not run after a stop keep zero scalars in the trace.
  if (trace)
    for (int64_t s = step; s < total_steps; ++s) trace[s] = hicu_trace{-1, -1, -1, 0, 0.0, 0.0, 0.0};
  HICU_HIP_TRY(wait.stream(st));
  return status;
}

}  // extern "C"
