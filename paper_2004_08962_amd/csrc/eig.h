#pragma once

#include "common.h"

namespace hicu {

size_t eig_workspace(int n);
// projector_only = false resolves every eigenvector to working accuracy
// (rotation floor 2e-15 of the largest diagonal entry, sweep test 1e-13);
// true is enough when only the projector onto the nullspace is used (floor
// 1e-13, the rounding level of the block updates, and sweep test 1e-9).
// Returns with the work queued on st (the public entry points wait).
int32_t run_eig(int n, int rank, const void* G, const void* V0, void* Q, double* evals, void* Vout,
                int32_t* sweeps_out, void* ws, size_t ws_bytes, hipStream_t st, bool projector_only);

}  // namespace hicu
