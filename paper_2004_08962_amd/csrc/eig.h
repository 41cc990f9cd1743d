#pragma once

#include "common.h"

namespace hicu {

size_t eig_workspace(int n);
int32_t run_eig(int n, int rank, const void* G, const void* V0, void* Q, double* evals, void* Vout,
                int32_t* sweeps_out, void* ws, size_t ws_bytes, hipStream_t st);

}  // namespace hicu
