// FP64 Hermitian eigendecomposition of the Gram matrix by two-sided block
// Jacobi on the device (nullspace update of Algorithm 1, Gram route of the
// DISCUSSION section).
//
// The matrix is split into 16-wide index blocks.  A sweep opens with one
// round over the block pairs (2j, 2j + 1) that rotates every index pair of
// each 32 x 32 subproblem (so every in-block pair is visited), then visits
// every pair of blocks once (round-robin "circle" schedule, nb - 1 rounds of
// nb/2 disjoint pairs) rotating only the 256 index pairs across the two
// blocks (16 inner rounds instead of 31): each index pair is rotated once
// per sweep.  In each round one workgroup per pair works on its subproblem
// with complex Jacobi rotations in LDS, and a second kernel applies the
// block-diagonal unitary W to the whole matrix and to the eigenvector
// accumulator (A <- W' A W, V <- V W) one 32 x 32 block per workgroup, in
// place.  Pairs that are already diagonal are skipped, so
// warm-started solves (the previous eigenvectors as V0) cost little.  A sweep
// ends with a relative off-diagonal test; FP64 throughout.
#include <algorithm>
#include <cmath>
#include <vector>

#include "eig.h"

namespace hicu {

constexpr int BS = 16;        // index block
constexpr int SB = 2 * BS;    // subproblem size
constexpr int MAX_INNER = 1;  // inner sweeps per subproblem (the outer sweeps finish the job)

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csc(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// Circle-method schedule: member t of round r among `cnt` players.
__device__ __forceinline__ int circle_pos(int t, int r, int cnt) {
  return t == 0 ? 0 : 1 + (t - 1 + r) % (cnt - 1);
}

struct Rot {
  double cs, sn;
  double2 e;   // unit phase of the off-diagonal entry
  int p, q;
  int did;     // rotation applied (otherwise identity)
};

// Rotation that diagonalises [[a, c], [conj(c), b]]: J = diag(1, conj(e)) R,
// R = [[cs, sn], [-sn, cs]], with t = sn/cs the smaller root of
// t^2 + 2 zeta t - 1 = 0, zeta = (b - a) / (2 |c|) (make_rot_fast below).

// B' = Ja^H B Jb for the 2x2 block B = [[b00, b01], [b10, b11]].
__device__ __forceinline__ void rot2x2(const Rot& ra, const Rot& rb, double2& b00, double2& b01, double2& b10,
                                       double2& b11) {
  // T = Ja^H B:  Ja^H = [[cs, -sn e], [sn, cs e]]
  const double2 ea = ra.e;
  const double2 t00 = cadd(csc(ra.cs, b00), csc(-ra.sn, cmul(ea, b10)));
  const double2 t01 = cadd(csc(ra.cs, b01), csc(-ra.sn, cmul(ea, b11)));
  const double2 t10 = cadd(csc(ra.sn, b00), csc(ra.cs, cmul(ea, b10)));
  const double2 t11 = cadd(csc(ra.sn, b01), csc(ra.cs, cmul(ea, b11)));
  // B' = T Jb:  Jb = [[cs, sn], [-sn conj(e), cs conj(e)]]
  const double2 eb = cconj(rb.e);
  b00 = cadd(csc(rb.cs, t00), csc(-rb.sn, cmul(t01, eb)));
  b01 = cadd(csc(rb.sn, t00), csc(rb.cs, cmul(t01, eb)));
  b10 = cadd(csc(rb.cs, t10), csc(-rb.sn, cmul(t11, eb)));
  b11 = cadd(csc(rb.sn, t10), csc(rb.cs, cmul(t11, eb)));
}

// Index blocks of pair `pair` in round r of the circle schedule; r < 0 is
// the sweep's opening round, which pairs blocks 2 pair and 2 pair + 1.
__device__ __forceinline__ void block_indices(int r, int nb, int pair, int* idx) {
  const int P = r < 0 ? 2 * pair : circle_pos(pair, r, nb), Q = r < 0 ? 2 * pair + 1 : circle_pos(nb - 1 - pair, r, nb);
  for (int i = 0; i < BS; ++i) {
    idx[i] = P * BS + i;
    idx[BS + i] = Q * BS + i;
  }
}

// Fast unitary-to-rounding rotation: reciprocal square roots and
// reciprocals from the hardware approximations plus one Newton step each.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  return y * (1.5 - 0.5 * x * y * y);
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * (2.0 - x * y);
  return y * (2.0 - x * y);
}

// With d = (b - a) / 2 and r = sqrt(d^2 + |c|^2): cos^2 = (1 + |d| / r) / 2,
// sin = |c| / (2 r cos), signed like d (the smaller rotation, |angle| <=
// pi/4); the phase of c goes into e.  Three reciprocal square roots, two of
// them independent, keep the dependent chain short.
__device__ __forceinline__ bool make_rot_fast(double a, double b, double2 c, double tol, double floor_abs, Rot* r) {
  const double c2 = c.x * c.x + c.y * c.y;
  r->cs = 1.0;
  r->sn = 0.0;
  r->e = make_double2(1.0, 0.0);
  if (!(c2 > tol * tol * fabs(a * b)) || !(c2 > floor_abs * floor_abs)) return false;
  const double d = 0.5 * (b - a);
  const double ir = rsqrt_nr(fma(d, d, c2));  // 1 / r
  const double ic = rsqrt_nr(c2);             // 1 / |c|
  const double cs2 = fma(0.5 * fabs(d), ir, 0.5);
  const double ics = rsqrt_nr(cs2);
  const double sn = 0.5 * c2 * ic * ir * ics;
  r->cs = cs2 * ics;
  r->sn = d >= 0.0 ? sn : -sn;
  r->e = make_double2(c.x * ic, c.y * ic);
  return true;
}

// One workgroup (1024 threads) per block pair: cyclic Jacobi on the 32x32
// subproblem in LDS, U written to Ubuf[pair].  Each inner round: 16 lanes
// compute the 16 rotations (skipping entries below the relative tolerance or
// the absolute noise floor), then every thread produces one element of the
// rotated S (double buffered) and one element of U.
__global__ __launch_bounds__(1024) void pair_eig_kernel(const double2* A, int npad, int nb, int round,
                                                        double tol, const double* floor_dev, double2* Ubuf,
                                                        int* ident) {
  __shared__ double2 S[2][SB][SB + 1];
  __shared__ double2 U[2][SB][SB + 1];
  __shared__ Rot rot[SB / 2];
  __shared__ int idx[SB];
  __shared__ int nrot_round, nrot_sweep[MAX_INNER];
  const int tid = threadIdx.x;
  const bool cross = round >= 0;
  if (tid == 0) block_indices(round, nb, blockIdx.x, idx);
  if (tid < MAX_INNER) nrot_sweep[tid] = 0;
  __syncthreads();
  {
    const int i = tid >> 5, j = tid & 31;
    S[0][i][j] = A[(size_t)idx[i] * npad + idx[j]];
    U[0][i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  const double fl = *floor_dev;
  // Early exit when no off-diagonal entry is above the rotation thresholds.
  __syncthreads();
  {
    const int i = tid >> 5, j = tid & 31;
    const double2 v = S[0][i][j];
    const double v2 = v.x * v.x + v.y * v.y;
    const bool active = cross ? ((i < BS) != (j < BS)) : i != j;
    const bool big = active && v2 > fl * fl && v2 > tol * tol * fabs(S[0][i][i].x * S[0][j][j].x);
    if (tid == 0) nrot_round = 0;
    __syncthreads();
    if (big) nrot_round = 1;
    __syncthreads();
    if (nrot_round == 0) {
      if (tid == 0) ident[blockIdx.x] = 1;
      return;
    }
  }
  // Threads 0..255 own one 2x2 block (al, be) of S (upper block triangle
  // only: S is Hermitian, the lower block is written as the mirror);
  // threads 256..767 own one row of U and one rotation pair (both
  // columns).  One thread per block reads each entry and rotation once,
  // which keeps the LDS traffic of a round low.
  const int al = tid >> 4, be = tid & 15;
  const int ut = tid - 256, ui = ut >> 4, ub = ut & 15;
  int cur = 0, total = 0;
  for (int sweep = 0; sweep < MAX_INNER; ++sweep) {
    for (int r = 0; r < (cross ? BS : SB - 1); ++r) {
      __syncthreads();
      if (tid < SB / 2) {
        // opening round: every pair of the 32 indices (circle schedule);
        // later rounds: only the pairs across the two blocks, whose
        // in-block pairs the opening round has rotated
        const int p = cross ? tid : circle_pos(tid, r, SB);
        const int q = cross ? BS + (tid + r) % BS : circle_pos(SB - 1 - tid, r, SB);
        Rot ro;
        const bool did = make_rot_fast(S[cur][p][p].x, S[cur][q][q].x, S[cur][p][q], tol, fl, &ro);
        ro.p = p;
        ro.q = q;
        ro.did = did;
        rot[tid] = ro;
        const uint64_t any = __ballot(did) & 0xffffull;
        if (tid == 0) {
          nrot_round = __popcll(any);
          nrot_sweep[sweep] += nrot_round;
        }
      }
      __syncthreads();
      if (nrot_round == 0) continue;  // uniform: nothing to rotate this round
      const int nx = cur ^ 1;
      if (tid < 256) {
        if (al <= be) {
          const Rot ra = rot[al], rb = rot[be];
          double2 b00 = S[cur][ra.p][rb.p], b01 = S[cur][ra.p][rb.q];
          double2 b10 = S[cur][ra.q][rb.p], b11 = S[cur][ra.q][rb.q];
          rot2x2(ra, rb, b00, b01, b10, b11);
          if (al == be) {
            if (ra.did) {
              b01 = b10 = make_double2(0.0, 0.0);
              b00.y = b11.y = 0.0;
            }
            S[nx][ra.p][ra.p] = b00;
            S[nx][ra.p][ra.q] = b01;
            S[nx][ra.q][ra.p] = b10;
            S[nx][ra.q][ra.q] = b11;
          } else {
            S[nx][ra.p][rb.p] = b00;
            S[nx][ra.p][rb.q] = b01;
            S[nx][ra.q][rb.p] = b10;
            S[nx][ra.q][rb.q] = b11;
            S[nx][rb.p][ra.p] = cconj(b00);
            S[nx][rb.q][ra.p] = cconj(b01);
            S[nx][rb.p][ra.q] = cconj(b10);
            S[nx][rb.q][ra.q] = cconj(b11);
          }
        }
      } else if (ut < SB * (SB / 2)) {
        // U <- U J for pair ub: new p = cs up - sn conj(e) uq,
        //                       new q = sn up + cs conj(e) uq
        const Rot ru = rot[ub];
        const double2 up = U[cur][ui][ru.p], uq = U[cur][ui][ru.q];
        const double2 w = cmul(uq, cconj(ru.e));
        U[nx][ui][ru.p] = cadd(csc(ru.cs, up), csc(-ru.sn, w));
        U[nx][ui][ru.q] = cadd(csc(ru.sn, up), csc(ru.cs, w));
      }
      cur = nx;
    }
    __syncthreads();
    const int nr = nrot_sweep[sweep];
    total += nr;
    if (nr == 0) break;
  }
  // A pair that needed no rotation keeps U = I; the apply step skips it.
  if (tid == 0) ident[blockIdx.x] = total == 0;
  if (total == 0) return;
  double2* out = Ubuf + (size_t)blockIdx.x * SB * SB;
  out[tid] = U[cur][tid >> 5][tid & 31];
}

// Workgroup (alpha, beta): A[ia, ib] <- Ua^H A[ia, ib] Ub and
// V[ia, ib] <- V[ia, ib] Ub, in place: the (alpha, beta) blocks partition
// both matrices, so each element is read and written by one workgroup only.
// Pairs whose subproblem needed no rotation have U = I and are skipped.
// 1024 threads, one output element each.  With `sums`, the workgroup also
// writes the squared Frobenius norms of the off-diagonal part and of its
// whole block (indices < n) for the convergence test.
__global__ __launch_bounds__(1024) void apply_kernel(double2* A, double2* V, int n, int npad, int nb, int round,
                                                     const double2* Ubuf, const int* ident, double* sums) {
  __shared__ double2 Bm[SB][SB + 1];
  __shared__ double2 Vm[SB][SB + 1];
  __shared__ double2 Ua[SB][SB + 1];
  __shared__ double2 Ub[SB][SB + 1];
  __shared__ int ia[SB], ib[SB];
  __shared__ double red[16];
  const int tid = threadIdx.x;
  const int alpha = blockIdx.x, beta = blockIdx.y;
  const bool ida = ident[alpha] != 0, idb = ident[beta] != 0;
  if (ida && idb && !sums) return;
  if (tid == 0) block_indices(round, nb, alpha, ia);
  if (tid == 1) block_indices(round, nb, beta, ib);
  __syncthreads();
  const int r = tid >> 5, c = tid & 31;
  const int gi = ia[r], gj = ib[c];
  double2 out = A[(size_t)gi * npad + gj];
  if (!(ida && idb)) {
    const double2* ua = Ubuf + (size_t)alpha * SB * SB;
    const double2* ub = Ubuf + (size_t)beta * SB * SB;
    Ua[r][c] = ida ? make_double2(r == c ? 1.0 : 0.0, 0.0) : ua[tid];
    Ub[r][c] = idb ? make_double2(r == c ? 1.0 : 0.0, 0.0) : ub[tid];
    Bm[r][c] = out;
    if (!idb) Vm[r][c] = V[(size_t)gi * npad + gj];
    __syncthreads();
    if (!ida) {  // T = Ua^H B
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll 8
      for (int k = 0; k < SB; ++k) acc = cadd(acc, cmulc(Ua[k][r], Bm[k][c]));
      out = acc;
      __syncthreads();
      Bm[r][c] = out;
      __syncthreads();
    }
    if (!idb) {  // out = T Ub, V <- V Ub
      double2 acc = make_double2(0.0, 0.0), vacc = make_double2(0.0, 0.0);
#pragma unroll 8
      for (int k = 0; k < SB; ++k) {
        acc = cadd(acc, cmul(Bm[r][k], Ub[k][c]));
        vacc = cadd(vacc, cmul(Vm[r][k], Ub[k][c]));
      }
      out = acc;
      V[(size_t)gi * npad + gj] = vacc;
    }
    A[(size_t)gi * npad + gj] = out;
  }
  if (sums) {
    double off2 = 0.0, all2 = 0.0;
    if (gi < n && gj < n) {
      all2 = out.x * out.x + out.y * out.y;
      if (gi != gj) off2 = all2;
    }
    off2 = block_sum_d(off2, red);
    all2 = block_sum_d(all2, red);
    if (tid == 0) {
      const size_t slot = (size_t)alpha * gridDim.y + beta;
      sums[2 * slot] = off2;
      sums[2 * slot + 1] = all2;
    }
  }
}

// Fixed-order sum of the per-block convergence partials: out = {off^2, all^2}.
__global__ __launch_bounds__(256) void sums_kernel(const double* part, int count, double* out) {
  __shared__ double red[4];
  double o = 0.0, a = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    o += part[2 * i];
    a += part[2 * i + 1];
  }
  o = block_sum_d(o, red);
  a = block_sum_d(a, red);
  if (threadIdx.x == 0) {
    out[0] = o;
    out[1] = a;
  }
}

// Absolute floor of the rotations: floor_rel times the largest diagonal
// entry of G.  With floor_rel = 2e-15 every eigenvector is resolved to
// working accuracy; 1e-13 is the rounding level of the 32-term block updates
// (about 32 eps times the largest eigenvalue), enough when only the
// projector onto the nullspace matters, and it lets converged pairs be
// skipped.
__global__ __launch_bounds__(256) void floor_kernel(const double2* G, int n, double floor_rel, double* out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, fabs(G[(size_t)i * n + i].x));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = floor_rel * red[0];
}

// A = G padded (identity on padding), V = I or V0 padded.
__global__ void init_kernel(const double2* G, const double2* V0, int n, int npad, double2* A, double2* V) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)npad * npad;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / npad), j = (int)(e % npad);
    const bool in = i < n && j < n;
    A[e] = in ? G[(size_t)i * n + j] : make_double2(i == j ? 1.0 : 0.0, 0.0);
    if (V0 && in) V[e] = V0[(size_t)i * n + j];
    else V[e] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
}

// C = op(X) Y for npad x npad complex matrices; op = conj-transpose when ct.
__global__ __launch_bounds__(256) void zgemm_kernel(const double2* X, const double2* Y, double2* C, int npad,
                                                    int ct) {
  __shared__ double2 Xs[32][33];
  __shared__ double2 Ys[32][33];
  const int tid = threadIdx.x;
  const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
  const int r = tid >> 3, c0 = (tid & 7) * 4;
  double2 acc[4];
  for (int c = 0; c < 4; ++c) acc[c] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < npad; k0 += 32) {
    for (int e = tid; e < 1024; e += 256) {
      const int i = e / 32, j = e % 32;
      // Xs[i][kk] = op(X)[bi + i][k0 + kk]
      Xs[i][j] = ct ? cconj(X[(size_t)(k0 + j) * npad + bi + i]) : X[(size_t)(bi + i) * npad + k0 + j];
      Ys[i][j] = Y[(size_t)(k0 + i) * npad + bj + j];
    }
    __syncthreads();
    for (int k = 0; k < 32; ++k) {
      const double2 xv = Xs[r][k];
      for (int c = 0; c < 4; ++c) acc[c] = cadd(acc[c], cmul(xv, Ys[k][c0 + c]));
    }
    __syncthreads();
  }
  for (int c = 0; c < 4; ++c) C[(size_t)(bi + r) * npad + bj + c0 + c] = acc[c];
}

// Ascending order of the n real eigenvalues (ties by index): perm[rank] = i.
__global__ void rank_kernel(const double2* A, int n, int npad, int* perm, double* vals) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double li = A[(size_t)i * npad + i].x;
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = A[(size_t)j * npad + j].x;
      rk += (lj < li) || (lj == li && j < i);
    }
    perm[rk] = i;
    vals[rk] = li;
  }
}

// One workgroup per output column: unit-phase normalisation (sum of entries
// real, >= 0) and scatter to Q (complex64) / Vout (complex128).
__global__ __launch_bounds__(256) void gather_kernel(const double2* V, int n, int npad, int nq, const int* perm,
                                                     float2* Q, double2* Vout) {
  __shared__ double red[4];
  const int col = blockIdx.x;
  const int src = perm[col];
  double sr = 0.0, si = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double2 v = V[(size_t)i * npad + src];
    sr += v.x;
    si += v.y;
  }
  sr = block_sum_d(sr, red);
  si = block_sum_d(si, red);
  __shared__ double2 ph;
  if (threadIdx.x == 0) {
    const double mg = sqrt(sr * sr + si * si);
    ph = mg > 0.0 ? make_double2(sr / mg, -si / mg) : make_double2(1.0, 0.0);
  }
  __syncthreads();
  const double2 p = ph;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double2 v = cmul(V[(size_t)i * npad + src], p);
    if (col < nq && Q) Q[(size_t)i * nq + col] = make_float2((float)v.x, (float)v.y);
    if (Vout) Vout[(size_t)i * n + col] = v;
  }
}

__global__ void copy_vals_kernel(const double* src, double* dst, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

static int npad_of(int n) { return (int)rup(n, SB); }

namespace {
struct EigLayout {
  size_t A, V, T, U, ident, part, perm, vals, sums, total;
};
EigLayout eig_layout(int n) {
  const size_t np = (size_t)npad_of(n), npair = np / SB;
  const size_t mat = np * np * sizeof(double2);
  EigLayout L;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += (b + 255) / 256 * 256;
    return o;
  };
  L.A = take(mat);
  L.V = take(mat);
  L.T = take(mat);
  L.U = take(npair * SB * SB * sizeof(double2));
  L.ident = take(npair * sizeof(int));
  L.part = take(2 * npair * npair * sizeof(double));
  L.perm = take(np * sizeof(int));
  L.vals = take(np * sizeof(double));
  L.sums = take(4 * sizeof(double));
  L.total = off;
  return L;
}
}  // namespace

size_t eig_workspace(int n) { return eig_layout(n).total; }

int32_t run_eig(int n, int rank, const void* G, const void* V0, void* Q, double* evals, void* Vout,
                int32_t* sweeps_out, void* ws, size_t ws_bytes, hipStream_t st, bool projector_only) {
  const double floor_rel = projector_only ? 1e-13 : 2e-15;
  const EigLayout L = eig_layout(n);
  if (ws == nullptr || ws_bytes < L.total) return HICU_ERR_WORKSPACE;
  const int np = npad_of(n), nb = np / BS, npair = nb / 2;
  const size_t mat = (size_t)np * np;
  char* base = reinterpret_cast<char*>(ws);
  double2* A = reinterpret_cast<double2*>(base + L.A);
  double2* V = reinterpret_cast<double2*>(base + L.V);
  double2* T = reinterpret_cast<double2*>(base + L.T);
  double2* Ub = reinterpret_cast<double2*>(base + L.U);
  int* ident = reinterpret_cast<int*>(base + L.ident);
  double* part = reinterpret_cast<double*>(base + L.part);
  int* perm = reinterpret_cast<int*>(base + L.perm);
  double* vals = reinterpret_cast<double*>(base + L.vals);
  double* dsums = reinterpret_cast<double*>(base + L.sums);
  double* dfloor = dsums + 2;
  const int gblocks = (int)std::min<int64_t>(cdiv((int64_t)mat, 256), 4096);
  hipLaunchKernelGGL(init_kernel, dim3(gblocks), dim3(256), 0, st, reinterpret_cast<const double2*>(G),
                     reinterpret_cast<const double2*>(V0), n, np, A, V);
  hipLaunchKernelGGL(floor_kernel, dim3(1), dim3(256), 0, st, reinterpret_cast<const double2*>(G), n, floor_rel,
                     dfloor);
  HICU_HIP_TRY(hipGetLastError());
  if (V0) {
    // A <- V0^H G V0 (the padding stays identity: V0 is padded with I).
    hipLaunchKernelGGL(zgemm_kernel, dim3(np / 32, np / 32), dim3(256), 0, st, V, A, T, np, 1);
    hipLaunchKernelGGL(zgemm_kernel, dim3(np / 32, np / 32), dim3(256), 0, st, T, V, A, np, 0);
    HICU_HIP_TRY(hipGetLastError());
  }
  // A sweep visits every block pair once.  Converged when the off-diagonal
  // Frobenius norm after a sweep is below tol of the whole, or when it has
  // reached the rounding floor (below 1e-10 and no longer halving per sweep).
  const double tol_inner = 1e-15, tol = projector_only ? 1e-9 : 1e-13, tol_floor = 1e-10;
  const int max_sweeps = 40;
  int sweeps = 0;
  double sums[2] = {0.0, 0.0}, prev = INFINITY;
  int32_t status = HICU_OK;
  for (;;) {
    // opening round: blocks (2 j, 2 j + 1) with all their index pairs
    hipLaunchKernelGGL(pair_eig_kernel, dim3(npair), dim3(1024), 0, st, (const double2*)A, np, nb, -1, tol_inner,
                       (const double*)dfloor, Ub, ident);
    hipLaunchKernelGGL(apply_kernel, dim3(npair, npair), dim3(1024), 0, st, A, V, n, np, nb, -1, (const double2*)Ub,
                       (const int*)ident, (double*)nullptr);
    for (int r = 0; r < nb - 1; ++r) {
      const bool last = r == nb - 2;
      hipLaunchKernelGGL(pair_eig_kernel, dim3(npair), dim3(1024), 0, st, (const double2*)A, np, nb, r, tol_inner,
                         (const double*)dfloor, Ub, ident);
      hipLaunchKernelGGL(apply_kernel, dim3(npair, npair), dim3(1024), 0, st, A, V, n, np, nb, r,
                         (const double2*)Ub, (const int*)ident, last ? part : nullptr);
    }
    hipLaunchKernelGGL(sums_kernel, dim3(1), dim3(256), 0, st, (const double*)part, npair * npair, dsums);
    HICU_HIP_TRY(hipGetLastError());
    ++sweeps;
    HICU_HIP_TRY(hipMemcpyAsync(sums, dsums, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HICU_HIP_TRY(hipStreamSynchronize(st));
    const double rel = sums[1] > 0.0 ? std::sqrt(sums[0] / sums[1]) : 0.0;
    if (!(rel == rel) || !std::isfinite(sums[1])) {
      status = HICU_ERR_NONFINITE;
      break;
    }
    if (rel <= tol || (rel <= tol_floor && rel > 0.5 * prev)) break;
    prev = rel;
    if (sweeps == max_sweeps) {
      status = HICU_ERR_NOCONV;
      break;
    }
  }
  if (sweeps_out) *sweeps_out = sweeps;
  if (status == HICU_ERR_NONFINITE) return status;
  hipLaunchKernelGGL(rank_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, (const double2*)A, n, np,
                     perm, vals);
  hipLaunchKernelGGL(gather_kernel, dim3(n), dim3(256), 0, st, (const double2*)V, n, np, n - rank,
                     (const int*)perm, reinterpret_cast<float2*>(Q), reinterpret_cast<double2*>(Vout));
  if (evals)
    hipLaunchKernelGGL(copy_vals_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, (const double*)vals,
                       evals, n);
  HICU_HIP_TRY(hipGetLastError());
  HICU_HIP_TRY(hipStreamSynchronize(st));
  return status;
}

}  // namespace hicu
