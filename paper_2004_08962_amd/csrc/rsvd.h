#pragma once

#include <algorithm>

#include "common.h"

namespace hicu {

// Sketch size l = ceil(3 r / 2), at most n.
inline int default_sketch(int rank, int n) { return std::min(n, (3 * rank + 1) / 2); }
// Largest n the Householder kernels hold per wave (32 complex values per lane).
constexpr int kRsvdMaxN = 2048;

size_t rsvd_workspace(const Geo& g, int rank, int ell);
// Q (complex64 n x (n - rank), row-major) orthogonal to the rank principal
// right singular vectors of the rSVD of H_S(x) with an l-column sketch drawn
// for (seed, outer, sid).  sv (optional, device) receives the l singular
// values of the sketched B, largest first; sweeps (optional, host) the
// Jacobi sweeps of its eigensolve.  basis = false resolves the singular
// vectors of B only to the eigensolver's projector accuracy (enough when
// only Q Q' is used); true resolves each of them, which fixes the
// Householder basis.  Returns with the work queued on st (the public entry
// point waits).
int32_t run_rsvd(const Geo& g, const void* x, int rank, int ell, uint64_t seed, uint32_t outer, uint32_t sid,
                 float2* Q, double* sv, int32_t* sweeps, void* ws, size_t ws_bytes, hipStream_t st, bool basis);

}  // namespace hicu
