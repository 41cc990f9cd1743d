// Tile-shape autotuner for the convolution kernels: candidates are timed on
// the caller's problem with HIP events and the fastest is kept in a
// process-wide cache consulted by every plan.
#pragma once

#include "common.h"
#include "conv.h"

namespace hicu {

struct TuneEntry {
  int tile;     // shape id (conv.h list)
  int chunk_c;  // adjoint channel chunk
  float ms;
};

// role 0: forward / line-search contraction (input = k-space, output = filters)
// role 1: adjoint contraction (input = residual, output = coils)
// roles 2, 3: the same for the batched runtime (shapes with batched kernels)
constexpr int kRoleBatchForward = 2, kRoleBatchAdjoint = 3;
bool tune_lookup(int role, int prec, const Geo& g, int p, TuneEntry* e);
void tune_store(int role, int prec, const Geo& g, int p, const TuneEntry& e);

}  // namespace hicu
