// FP64 Hermitian eigendecomposition of the Gram matrix by two-sided block
// Jacobi on the device (nullspace update of Algorithm 1, Gram route of the
// DISCUSSION section).
//
// The matrix is split into 16-wide index blocks; a sweep visits every pair of
// blocks once (round-robin "circle" schedule, nb - 1 rounds of nb/2 disjoint
// pairs).  In each round one workgroup per pair diagonalises its 32 x 32
// Hermitian subproblem with cyclic complex Jacobi rotations in LDS, and a
// second kernel applies the block-diagonal unitary W to the whole matrix and
// to the eigenvector accumulator (A <- W' A W, V <- V W) one 32 x 32 block per
// workgroup, ping-ponging between two buffers.  A sweep ends with a relative
// off-diagonal test; FP64 throughout.
#include <algorithm>
#include <cmath>
#include <vector>

#include "eig.h"

namespace hicu {

constexpr int BS = 16;        // index block
constexpr int SB = 2 * BS;    // subproblem size
constexpr int MAX_INNER = 12; // inner sweeps per subproblem

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
};

// Rotation that diagonalises [[a, c], [conj(c), b]]: J = diag(1, conj(e)) R,
// R = [[cs, sn], [-sn, cs]], with t = sn/cs the smaller root of
// t^2 + 2 zeta t - 1 = 0, zeta = (b - a) / (2 |c|).
// Entries below tol * sqrt(|a b|) or below the absolute floor (the rounding
// level of the subproblem) are left alone.
__device__ __forceinline__ bool make_rot(double a, double b, double2 c, double tol, double floor_abs, Rot* r) {
  const double ac = sqrt(c.x * c.x + c.y * c.y);
  r->cs = 1.0;
  r->sn = 0.0;
  r->e = make_double2(1.0, 0.0);
  if (!(ac > tol * sqrt(fabs(a * b))) || !(ac > floor_abs)) return false;
  const double zeta = (b - a) / (2.0 * ac);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  r->cs = 1.0 / sqrt(1.0 + t * t);
  r->sn = t * r->cs;
  r->e = make_double2(c.x / ac, c.y / ac);
  return true;
}

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

__device__ __forceinline__ void block_indices(int r, int nb, int pair, int* idx) {
  const int P = circle_pos(pair, r, nb), Q = circle_pos(nb - 1 - pair, r, nb);
  for (int i = 0; i < BS; ++i) {
    idx[i] = P * BS + i;
    idx[BS + i] = Q * BS + i;
  }
}

// One workgroup per block pair: full eigendecomposition of the 32x32
// subproblem, U written to Ubuf[pair].
__global__ __launch_bounds__(256) void pair_eig_kernel(const double2* A, int npad, int nb, int round,
                                                       double tol, double2* Ubuf) {
  __shared__ double2 S[SB][SB + 1];
  __shared__ double2 U[SB][SB + 1];
  __shared__ Rot rot[SB / 2];
  __shared__ int idx[SB];
  __shared__ int nrot;
  __shared__ double floor_abs;
  const int tid = threadIdx.x;
  if (tid == 0) block_indices(round, nb, blockIdx.x, idx);
  __syncthreads();
  for (int e = tid; e < SB * SB; e += 256) {
    const int i = e / SB, j = e % SB;
    S[i][j] = A[(size_t)idx[i] * npad + idx[j]];
    U[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  if (tid == 0) {
    double md = 0.0;
    for (int i = 0; i < SB; ++i) md = fmax(md, fabs(S[i][i].x));
    floor_abs = 4e-16 * md;
  }
  __syncthreads();
  for (int sweep = 0; sweep < MAX_INNER; ++sweep) {
    if (tid == 0) nrot = 0;
    __syncthreads();
    for (int r = 0; r < SB - 1; ++r) {
      if (tid < SB / 2) {
        const int p = circle_pos(tid, r, SB), q = circle_pos(SB - 1 - tid, r, SB);
        Rot ro;
        const bool did = make_rot(S[p][p].x, S[q][q].x, S[p][q], tol, floor_abs, &ro);
        ro.p = p;
        ro.q = q;
        rot[tid] = ro;
        if (did) atomicAdd(&nrot, 1);
      }
      __syncthreads();
      {
        const Rot ra = rot[tid >> 4], rb = rot[tid & 15];
        double2 b00 = S[ra.p][rb.p], b01 = S[ra.p][rb.q], b10 = S[ra.q][rb.p], b11 = S[ra.q][rb.q];
        rot2x2(ra, rb, b00, b01, b10, b11);
        if ((tid >> 4) == (tid & 15)) {
          b01 = make_double2(0.0, 0.0);
          b10 = make_double2(0.0, 0.0);
          b00.y = 0.0;
          b11.y = 0.0;
        }
        S[ra.p][rb.p] = b00;
        S[ra.p][rb.q] = b01;
        S[ra.q][rb.p] = b10;
        S[ra.q][rb.q] = b11;
      }
      for (int e = tid; e < SB * (SB / 2); e += 256) {
        const int i = e / (SB / 2);
        const Rot rb = rot[e % (SB / 2)];
        const double2 up = U[i][rb.p], uq = U[i][rb.q];
        const double2 eb = cconj(rb.e);
        U[i][rb.p] = cadd(csc(rb.cs, up), csc(-rb.sn, cmul(uq, eb)));
        U[i][rb.q] = cadd(csc(rb.sn, up), csc(rb.cs, cmul(uq, eb)));
      }
      __syncthreads();
    }
    if (nrot == 0) break;
    __syncthreads();
  }
  double2* out = Ubuf + (size_t)blockIdx.x * SB * SB;
  for (int e = tid; e < SB * SB; e += 256) out[e] = U[e / SB][e % SB];
}

// Workgroup (alpha, beta): A'[ia, ib] = Ua^H A[ia, ib] Ub and
// V'[ia, ib] = V[ia, ib] Ub (rows ia cover every row once over alpha).
__global__ __launch_bounds__(256) void apply_kernel(const double2* A, double2* An, const double2* V,
                                                    double2* Vn, int npad, int nb, int round,
                                                    const double2* Ubuf) {
  __shared__ double2 Bm[SB][SB + 1];
  __shared__ double2 Ua[SB][SB + 1];
  __shared__ double2 Ub[SB][SB + 1];
  __shared__ int ia[SB], ib[SB];
  const int tid = threadIdx.x;
  const int alpha = blockIdx.x, beta = blockIdx.y;
  if (tid == 0) block_indices(round, nb, alpha, ia);
  if (tid == 1) block_indices(round, nb, beta, ib);
  __syncthreads();
  const double2* ua = Ubuf + (size_t)alpha * SB * SB;
  const double2* ub = Ubuf + (size_t)beta * SB * SB;
  for (int e = tid; e < SB * SB; e += 256) {
    const int i = e / SB, j = e % SB;
    Ua[i][j] = ua[e];
    Ub[i][j] = ub[e];
    Bm[i][j] = A[(size_t)ia[i] * npad + ib[j]];
  }
  __syncthreads();
  const int r = tid >> 3, c0 = (tid & 7) * 4;
  double2 t[4];
  for (int c = 0; c < 4; ++c) {
    double2 s = make_double2(0.0, 0.0);
    for (int k = 0; k < SB; ++k) s = cadd(s, cmulc(Ua[k][r], Bm[k][c0 + c]));
    t[c] = s;
  }
  __syncthreads();
  for (int c = 0; c < 4; ++c) Bm[r][c0 + c] = t[c];
  __syncthreads();
  for (int c = 0; c < 4; ++c) {
    double2 s = make_double2(0.0, 0.0);
    for (int k = 0; k < SB; ++k) s = cadd(s, cmul(Bm[r][k], Ub[k][c0 + c]));
    An[(size_t)ia[r] * npad + ib[c0 + c]] = s;
  }
  __syncthreads();
  for (int e = tid; e < SB * SB; e += 256) {
    const int i = e / SB, j = e % SB;
    Bm[i][j] = V[(size_t)ia[i] * npad + ib[j]];
  }
  __syncthreads();
  for (int c = 0; c < 4; ++c) {
    double2 s = make_double2(0.0, 0.0);
    for (int k = 0; k < SB; ++k) s = cadd(s, cmul(Bm[r][k], Ub[k][c0 + c]));
    Vn[(size_t)ia[r] * npad + ib[c0 + c]] = s;
  }
}

// Squared Frobenius norms of the off-diagonal part and of the whole matrix
// (indices < n), reduced in a fixed order: out[0] = off^2, out[1] = total^2.
__global__ __launch_bounds__(1024) void offdiag_kernel(const double2* A, int n, int npad, double* out) {
  __shared__ double red[16];
  double off = 0.0, tot = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    const double2 v = A[(size_t)i * npad + j];
    const double a2 = v.x * v.x + v.y * v.y;
    tot += a2;
    if (i != j) off += a2;
  }
  off = block_sum_d(off, red);
  tot = block_sum_d(tot, red);
  if (threadIdx.x == 0) {
    out[0] = off;
    out[1] = tot;
  }
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

size_t eig_workspace(int n) {
  const size_t np = (size_t)npad_of(n);
  const size_t mat = np * np * sizeof(double2);
  const size_t ub = (np / SB) * SB * SB * sizeof(double2);
  return 4 * mat + ub + np * (sizeof(int) + sizeof(double)) + 4096;
}

int32_t run_eig(int n, int rank, const void* G, const void* V0, void* Q, double* evals, void* Vout,
                int32_t* sweeps_out, void* ws, size_t ws_bytes, hipStream_t st) {
  if (ws == nullptr || ws_bytes < eig_workspace(n)) return HICU_ERR_WORKSPACE;
  const int np = npad_of(n), nb = np / BS;
  const size_t mat = (size_t)np * np;
  double2* A0 = reinterpret_cast<double2*>(ws);
  double2* A1 = A0 + mat;
  double2* Va = A1 + mat;
  double2* Vb = Va + mat;
  double2* Ub = Vb + mat;
  int* perm = reinterpret_cast<int*>(Ub + (size_t)(np / SB) * SB * SB);
  double* vals = reinterpret_cast<double*>(perm + np);
  double* offv = vals + np;
  const int gblocks = (int)std::min<int64_t>(cdiv((int64_t)mat, 256), 4096);
  hipLaunchKernelGGL(init_kernel, dim3(gblocks), dim3(256), 0, st, reinterpret_cast<const double2*>(G),
                     reinterpret_cast<const double2*>(V0), n, np, A0, Va);
  HICU_HIP_TRY(hipGetLastError());
  double2 *A = A0, *An = A1, *V = Va, *Vn = Vb;
  if (V0) {
    // A <- V0^H G V0 (padding stays identity since V0 is padded with I).
    hipLaunchKernelGGL(zgemm_kernel, dim3(np / 32, np / 32), dim3(256), 0, st, V, A, An, np, 1);
    hipLaunchKernelGGL(zgemm_kernel, dim3(np / 32, np / 32), dim3(256), 0, st, An, V, A, np, 0);
    HICU_HIP_TRY(hipGetLastError());
  }
  // Converged when the off-diagonal Frobenius norm is below 1e-13 of the
  // whole, or when it has reached the rounding floor (below 1e-10 and no
  // longer halving per sweep).
  const double tol_inner = 1e-15, tol = 1e-13, tol_floor = 1e-10;
  const int max_sweeps = 40;
  int sweeps = 0;
  double sums[2] = {0.0, 0.0}, prev = INFINITY;
  int32_t status = HICU_OK;
  for (;;) {
    hipLaunchKernelGGL(offdiag_kernel, dim3(1), dim3(1024), 0, st, A, n, np, offv);
    HICU_HIP_TRY(hipGetLastError());
    HICU_HIP_TRY(hipMemcpyAsync(sums, offv, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
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
    for (int r = 0; r < nb - 1; ++r) {
      hipLaunchKernelGGL(pair_eig_kernel, dim3(nb / 2), dim3(256), 0, st, (const double2*)A, np, nb, r,
                         tol_inner, Ub);
      hipLaunchKernelGGL(apply_kernel, dim3(nb / 2, nb / 2), dim3(256), 0, st, (const double2*)A, An,
                         (const double2*)V, Vn, np, nb, r, (const double2*)Ub);
      std::swap(A, An);
      std::swap(V, Vn);
    }
    HICU_HIP_TRY(hipGetLastError());
    ++sweeps;
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
