// Autotuner: times every valid tile shape of the forward and adjoint
// contractions on the caller's problem and caches the fastest per
// (role, precision, kernel box, coils, filters, size class).
#include "tune.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "step.h"

namespace hicu {
namespace {

std::mutex mu;
std::map<std::string, TuneEntry> cache;

std::string key_of(int role, int prec, const Geo& g, int p) {
  char buf[160];
  const int size_class = (int)std::floor(std::log2((double)std::max<int64_t>(1, g.s)));
  std::snprintf(buf, sizeof(buf), "r%d/q%d/k%dx%dx%d/c%d/p%d/s%d/d%d", role, prec, g.k[0], g.k[1], g.k[2], g.nc, p,
                size_class, g.d[0] > 1 ? 3 : 2);
  return buf;
}

// A shape is a candidate when it fits the problem's dimensionality (T0 > 1
// only with a kernel extent above 1 on axis 0) and, for D > 1, packs
// outputs of a kernel with at least 3 taps on axis 2; for the batched
// runtime only shapes with a persistent batched kernel qualify, and not
// the k-split ones: timed on one slice they won, but over the 64 uneven
// slices of the batched workload the batched BF16 adjoint with KS = 2 took
// 0.84 ms against 0.73 ms for 1 x 16 x 16 with two column fragments.
bool candidate(const Geo& g, int tile, bool batched) {
  const TileCfg t = tile_cfg(tile);
  if (g.k[0] == 1 && g.m[0] <= 1 && t.T0 > 1) return false;
  if (t.D > 1 && g.k[2] < 3) return false;
  if (batched && (!tile_batch_ok(tile) || t.KS > 1)) return false;
  return true;
}

// Median-free timing: one warm launch, then the mean of `reps` launches.
int32_t time_plan(const ConvPlan& p, hipStream_t st, float* ms) {
  hipEvent_t a, b;
  HICU_HIP_TRY(hipEventCreate(&a));
  HICU_HIP_TRY(hipEventCreate(&b));
  int32_t s = launch_conv(p, st);
  const int reps = 3;
  if (s == HICU_OK) {
    (void)hipEventRecord(a, st);
    for (int i = 0; i < reps && s == HICU_OK; ++i) s = launch_conv(p, st);
    (void)hipEventRecord(b, st);
    (void)hipEventSynchronize(b);
    float t = 0.f;
    (void)hipEventElapsedTime(&t, a, b);
    *ms = t / reps;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return s;
}

}  // namespace

bool tune_lookup(int role, int prec, const Geo& g, int p, TuneEntry* e) {
  std::lock_guard<std::mutex> l(mu);
  auto it = cache.find(key_of(role, prec, g, p));
  if (it == cache.end()) return false;
  *e = it->second;
  return true;
}

void tune_store(int role, int prec, const Geo& g, int p, const TuneEntry& e) {
  std::lock_guard<std::mutex> l(mu);
  cache[key_of(role, prec, g, p)] = e;
}

// Filters timed at once: one filter group of the gradient (the whole p when
// Y fits the residual budget), so the tuner needs no more memory than a
// step.  Per-column work is the same in every group, so a group ranks the
// shapes as the whole launch would.
static int tune_group(const Geo& g, int p) { return filter_group(g.s, p); }

static size_t tune_weights(const Geo& g, int p, int prec) {
  size_t wmax = 0;
  for (int cc : {16, 8, 4})
    for (int D : {1, 2, 4})
      wmax = std::max(wmax, weight_shape(prec, g.k, p, std::min(cc, p), 2 * g.nc, D).elems);
  return std::max(wmax, weight_shape(prec, g.k, g.nc, g.nc, 2 * p, 1).elems);
}

// Workspace of the tuner: Y of one filter group, a gradient buffer, the
// largest weight set and the largest partial-sum array over the candidates.
size_t tune_workspace(const Geo& g, int p, int prec) {
  const int pg = tune_group(g, p);
  const size_t wmax = tune_weights(g, p, prec);
  const int64_t ext = region_points(g);
  const int64_t blocks = (int64_t)(cdiv(ext, 16) + 1) * 4 * cdiv(std::max(2 * pg, 8 * g.nc), 16);
  return al((size_t)g.s * pg * sizeof(float2)) + al((size_t)g.npts * g.nc * sizeof(float2)) +
         2 * al(wmax * esize(prec)) + al((size_t)blocks * sizeof(double));
}

int32_t autotune(const Geo& g, const void* x, const void* F, int p, int prec, void* ws, size_t ws_bytes,
                 hipStream_t st, TuneEntry* best_fwd, TuneEntry* best_adj, bool batched) {
  const int role_f = batched ? kRoleBatchForward : 0, role_a = batched ? kRoleBatchAdjoint : 1;
  if (ws == nullptr || ws_bytes < tune_workspace(g, p, prec)) return HICU_ERR_WORKSPACE;
  const int pg = tune_group(g, p);
  size_t off = 0;
  float2* Y = reinterpret_cast<float2*>(at(ws, off));
  off += al((size_t)g.s * pg * sizeof(float2));
  float2* gbuf = reinterpret_cast<float2*>(at(ws, off));
  off += al((size_t)g.npts * g.nc * sizeof(float2));
  const size_t wmax = tune_weights(g, p, prec);
  void* B = at(ws, off);
  off += al(wmax * esize(prec));
  void* Blo = at(ws, off);
  off += al(wmax * esize(prec));
  double* part = reinterpret_cast<double*>(at(ws, off));
  const float2* Fc = reinterpret_cast<const float2*>(F);

  // forward over the first pg filters, Y stored s x pg
  StepPlan sp;
  HICU_TRY(make_step_plan(g, p, prec, false, &sp));
  HICU_TRY(launch_prep_weights(0, prec, g, Fc, p, sp.wf, B, Blo, st));
  auto group_forward = [&](ConvPlan& c) {
    sp.cf = c;
    fill_forward_args(g, x, sp, ws, reinterpret_cast<float*>(Y), part);
    c = sp.cf;
    c.a.B = B;
    c.a.Blo = Blo;
    c.a.coutr = 2 * pg;
    c.a.os[0] = g.m[1] * g.m[2] * pg;
    c.a.os[1] = g.m[2] * pg;
    c.a.os[2] = pg;
    c.gy = (int)cdiv(2 * pg, block_cols(c.t));
  };
  TuneEntry bf{-1, g.nc, 1e30f};
  for (int tile = 0; tile < kNumTiles; ++tile) {
    if (!candidate(g, tile, batched) || tile_D(tile) != 1) continue;
    ConvPlan cp;
    if (plan_conv(prec, tile, g.k, sp.wf, sp.wf.nchunks, g.m, 2 * p, &cp) != HICU_OK) continue;
    group_forward(cp);
    float ms = 0.f;
    if (time_plan(cp, st, &ms) != HICU_OK) continue;
    if (ms < bf.ms) bf = TuneEntry{tile, g.nc, ms};
  }
  if (bf.tile < 0) return HICU_ERR_UNSUPPORTED;
  tune_store(role_f, prec, g, p, bf);
  // Y of the group from the chosen shape, as the adjoint's input
  {
    ConvPlan cp;
    HICU_TRY(plan_conv(prec, bf.tile, g.k, sp.wf, sp.wf.nchunks, g.m, 2 * p, &cp));
    group_forward(cp);
    HICU_TRY(launch_conv(cp, st));
  }

  // adjoint of the group
  const int64_t oe[3] = {g.hi[0] - g.lo[0], g.hi[1] - g.lo[1], g.hi[2] - g.lo[2]};
  TuneEntry ba{-1, 0, 1e30f};
  for (int D : {1, 2, 4}) {
    for (int cc : {16, 8, 4}) {
      const int chunk = std::min(cc, p);
      const WeightShape wa = weight_shape(prec, g.k, p, chunk, 2 * g.nc, D);
      bool built = false;
      for (int tile = 0; tile < kNumTiles; ++tile) {
        if (!candidate(g, tile, batched) || tile_D(tile) != D) continue;
        ConvPlan cp;
        if (plan_conv(prec, tile, g.k, wa, wa.nchunks, oe, 2 * g.nc, &cp) != HICU_OK) continue;
        if (!built) {
          HICU_TRY(launch_prep_weights(1, prec, g, Fc, p, wa, B, Blo, st));
          built = true;
        }
        fill_adjoint_args(g, Y, pg, B, Blo, gbuf, nullptr, part, cp.a);
        cp.a.nchunks = (int)cdiv(pg, chunk);
        float ms = 0.f;
        if (time_plan(cp, st, &ms) != HICU_OK) continue;
        if (ms < ba.ms) ba = TuneEntry{tile, chunk, ms};
      }
      if (chunk < cc) break;
    }
  }
  if (ba.tile < 0) return HICU_ERR_UNSUPPORTED;
  tune_store(role_a, prec, g, p, ba);
  if (best_fwd) *best_fwd = bf;
  if (best_adj) *best_adj = ba;
  HICU_HIP_TRY(hipStreamSynchronize(st));
  return HICU_OK;
}

}  // namespace hicu

using namespace hicu;

extern "C" {

size_t hicu_autotune_workspace_bytes(const hicu_geom* gm, int32_t p, int32_t prec) {
  Geo g;
  if (make_geo(gm, &g) != HICU_OK || p < 1 || !valid_prec(prec)) return 0;
  return tune_workspace(g, p, prec);
}

static int32_t autotune_entry(const hicu_geom* gm, const void* x, const void* F, int32_t p, int32_t prec, void* ws,
                              size_t ws_bytes, int32_t* choice, void* stream, bool batched) {
  Geo g;
  HICU_TRY(make_geo(gm, &g));
  if (!x || !F || !valid_prec(prec)) return HICU_ERR_ARG;
  if (p < 1 || p > 1 << 20) return HICU_ERR_RANK;
  if (g.wrap[0] || g.wrap[1] || g.wrap[2] || g.kmasked) return HICU_ERR_UNSUPPORTED;
  if (batched && prec == P_F16) return HICU_ERR_UNSUPPORTED;
  TuneEntry f, a;
  HICU_TRY(autotune(g, x, F, p, prec, ws, ws_bytes, (hipStream_t)stream, &f, &a, batched));
  if (choice) {
    const int32_t c[4] = {f.tile, f.chunk_c, a.tile, a.chunk_c};
    std::memcpy(choice, c, sizeof(c));
  }
  return HICU_OK;
}

int32_t hicu_autotune(const hicu_geom* gm, const void* x, const void* F, int32_t p, int32_t prec, void* ws,
                      size_t ws_bytes, int32_t* choice, void* stream) {
  return autotune_entry(gm, x, F, p, prec, ws, ws_bytes, choice, stream, false);
}

int32_t hicu_autotune_batched(const hicu_geom* gm, const void* x, const void* F, int32_t p, int32_t prec, void* ws,
                              size_t ws_bytes, int32_t* choice, void* stream) {
  return autotune_entry(gm, x, F, p, prec, ws, ws_bytes, choice, stream, true);
}

int32_t hicu_tune_save(const char* path) {
  if (!path) return HICU_ERR_ARG;
  std::lock_guard<std::mutex> l(mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return HICU_ERR_ARG;
  for (const auto& kv : cache)
    std::fprintf(f, "%s %d %d %.6f\n", kv.first.c_str(), kv.second.tile, kv.second.chunk_c, kv.second.ms);
  std::fclose(f);
  return HICU_OK;
}

int32_t hicu_tune_load(const char* path) {
  if (!path) return HICU_ERR_ARG;
  FILE* f = std::fopen(path, "r");
  if (!f) return HICU_ERR_ARG;
  char key[160];
  TuneEntry e;
  int n = 0;
  std::lock_guard<std::mutex> l(mu);
  while (std::fscanf(f, "%159s %d %d %f", key, &e.tile, &e.chunk_c, &e.ms) == 4) {
    const bool ok = e.tile >= 0 && e.tile < kNumTiles && e.chunk_c >= 1;
    if (ok) {
      cache[key] = e;
      ++n;
    }
  }
  std::fclose(f);
  return n;
}

int32_t hicu_tune_put(const hicu_geom* gm, int32_t p, int32_t prec, int32_t role, int32_t tile, int32_t chunk_c) {
  Geo g;
  HICU_TRY(make_geo(gm, &g));
  if (!valid_prec(prec) || role < 0 || role > 3 || p < 1) return HICU_ERR_ARG;
  if (tile < 0 || tile >= kNumTiles || chunk_c < 1) return HICU_ERR_ARG;
  if ((role == 0 || role == 2) && tile_D(tile) != 1) return HICU_ERR_ARG;
  if (role >= 2 && !tile_batch_ok(tile)) return HICU_ERR_ARG;
  tune_store(role, prec, g, p, TuneEntry{tile, chunk_c, 0.f});
  return HICU_OK;
}

int32_t hicu_tile_count(void) { return kNumTiles; }

int32_t hicu_tile_info(int32_t tile, int32_t* cfg) {
  if (tile < 0 || tile >= kNumTiles || !cfg) return HICU_ERR_ARG;
  const TileCfg t = tile_cfg(tile);
  cfg[0] = t.T0;
  cfg[1] = t.T2;
  cfg[2] = t.WC;
  cfg[3] = t.FN;
  cfg[4] = t.D;
  cfg[5] = t.KS;
  return HICU_OK;
}

int32_t hicu_tune_clear(void) {
  std::lock_guard<std::mutex> l(mu);
  cache.clear();
  return HICU_OK;
}

}  // extern "C"
