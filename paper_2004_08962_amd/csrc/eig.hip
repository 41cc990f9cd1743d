// FP64 Hermitian eigendecomposition of the Gram matrix by two-sided block
// Jacobi on the device (nullspace update of Algorithm 1, Gram route of the
// DISCUSSION section).
//
// The matrix is split into 16-wide index blocks.  A sweep opens with one
// round over the block pairs (2j, 2j + 1) that rotates the index pairs
// inside each block (so every in-block pair is visited), then visits every
// pair of blocks once (round-robin "circle" schedule, nb - 1 rounds of nb/2
// disjoint pairs) rotating the 256 index pairs across the two blocks: each
// index pair is rotated once per sweep.  The opening round's subproblems are solved in LDS by
// pair_eig_kernel.  Each later round is one round_kernel launch: its first
// workgroups solve that round's subproblems (blocks formed from the
// previous round's results, rotations with the subproblem in registers)
// while the others apply the previous round's block-diagonal unitary W to
// the matrix and to the eigenvector accumulator (A <- W' A W into the
// other of two buffers, V <- V W in place) on the FP64 matrix cores.
// Pairs whose subproblem needs no rotation are flagged and their update is
// a copy, so warm-started solves (the previous eigenvectors as V0) cost
// little.  A sweep ends with a relative off-diagonal test; FP64
// throughout.
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

// Fast unitary-to-rounding rotation: reciprocal square roots from the
// hardware approximation (about 2^-24 relative) plus two Newton steps
// (2^-52; one step leaves 2^-48).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  return y * (1.5 - 0.5 * x * y * y);
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
// subproblem in LDS, U written to Ubuf[pair]; the opening round rotates
// the in-block pairs of both blocks (15 inner rounds).  Each inner round: 16 lanes
// compute the 16 rotations (skipping entries below the relative tolerance or
// the absolute noise floor), then every thread produces one element of the
// rotated S (double buffered) and one element of U.  Sfin[pair] receives
// the final diagonal 16-blocks of the subproblem.
__global__ __launch_bounds__(1024) void pair_eig_kernel(const double2* A, int npad, int nb, int round,
                                                        double tol, const double* floor_dev, double2* Ubuf,
                                                        int* ident, double2* Sfin) {
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
    const bool active = cross ? ((i < BS) != (j < BS)) : ((i < BS) == (j < BS) && i != j);
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
    for (int r = 0; r < (cross ? BS : BS - 1); ++r) {
      __syncthreads();
      if (tid < SB / 2) {
        // opening round: the pairs inside each of the two blocks (a circle
        // schedule on 16 indices per block, 8 rotations each); the pairs
        // across two blocks are rotated in the circle round that pairs
        // those blocks (cross rounds: t with BS + (t + r) mod BS)
        const int blk = tid >> 3, tt = tid & 7;
        const int p = cross ? tid : blk * BS + circle_pos(tt, r, BS);
        const int q = cross ? BS + (tid + r) % BS : blk * BS + circle_pos(BS - 1 - tt, r, BS);
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
  // final diagonal 16-blocks of the subproblem, for the next round's pairs
  if (tid < 512) {
    const int blk = tid >> 8, i = (tid >> 4) & 15, j = tid & 15;
    Sfin[(size_t)blockIdx.x * 512 + tid] = S[cur][blk * BS + i][blk * BS + j];
  }
}

// Index i (0..31) of pair `pair` in round r: its first 16-block, then its second.
__device__ __forceinline__ int pair_index(int r, int nb, int pair, int i) {
  const int P = r < 0 ? 2 * pair : circle_pos(pair, r, nb), Q = r < 0 ? 2 * pair + 1 : circle_pos(nb - 1 - pair, r, nb);
  return i < BS ? P * BS + i : Q * BS + (i - BS);
}

// The pair holding 16-block X in round r and X's offset in it (0 or BS):
// the inverse of the circle schedule.
__device__ __forceinline__ void block_owner(int r, int nb, int X, int* pair, int* off) {
  if (r < 0) {
    *pair = X >> 1;
    *off = (X & 1) * BS;
    return;
  }
  const int m = nb - 1;
  const int t = X == 0 ? 0 : 1 + (((X - 1 - r) % m) + m) % m;
  *pair = t < nb / 2 ? t : nb - 1 - t;
  *off = t < nb / 2 ? 0 : BS;
}

constexpr int kRoundThreads = 256;
constexpr size_t kRoundLds = 56 * 1024;

// Pair role of a round launch: solve round r's subproblem of pair `pair`
// (blocks P, Q) without waiting for round r - 1's update of A.  Its four
// 16 x 16 blocks of A^(r) = W'A^(r-1)W are formed here: the diagonal ones
// are the final subproblem matrices of the round r - 1 pairs that held P
// and Q (or A^(r-1) itself where such a pair did not rotate), the block
// (P, Q) is Ux' A^(r-1)[I_x, I_y] Uy with I_x, I_y the index sets of those
// pairs and Ux, Uy the 16 columns of their U that map to P and Q.
//
// The cross rotations then run with the subproblem in registers: thread
// (a, b) = (tid / 16, tid % 16) holds the 2x2 block on rows (P a, Q s(a))
// and columns (P b, Q s(b)), s(x) = (x + k) mod 16 at inner round k, so
// that rotation t of round k (indices P t and Q s(t)) acts on thread row t
// and thread column t only; between inner rounds s advances by one and the
// Q parts move one thread row / column through LDS.  Thread (a, b) also
// holds U[i][P a] and U[i][Q s(a)] for rows i = b, b + 16, so it needs
// rotations a and b only: it forms rotation b from the published diagonal
// blocks and reads rotation a from a lane of its wave (one barrier per
// inner round).  Outputs: U (unless no
// rotation was needed), the identity flag, and the final diagonal
// 16-blocks for the next round.
__device__ void pair_role(const double2* Ain, int npad, int nb, int r, int pair, const double2* Ucur,
                          const int* idcur, const double2* Scur, double2* Unext, int* idnext, double2* Snext,
                          double tol, double fl, unsigned char* lds) {
  const int tid = threadIdx.x;
  const int a = tid >> 4, b = tid & 15;
  const int P = circle_pos(pair, r, nb), Q = circle_pos(nb - 1 - pair, r, nb);
  int pp, op, pq, oq;
  block_owner(r - 1, nb, P, &pp, &op);
  block_owner(r - 1, nb, Q, &pq, &oq);
  // Every operand is loaded before the identity flags are known (the U and
  // final-block buffers of a pair that did not rotate hold stale but
  // in-bounds values, replaced below), so the loads overlap.
  const int idp_raw = idcur[pp], idq_raw = idcur[pq];
  double2 stt, sbb, stb, sbt;
  {
    auto M = reinterpret_cast<double2(*)[SB + 1]>(lds);                       // 32 x 33
    auto Ux = reinterpret_cast<double2(*)[BS + 1]>(lds + 32 * 33 * 16);       // 32 x 17
    auto Uy = reinterpret_cast<double2(*)[BS + 1]>(lds + 32 * 50 * 16);       // 32 x 17
    auto LP = reinterpret_cast<double2(*)[SB][BS + 1]>(lds + 32 * 67 * 16);   // 2 x 32 x 17
    auto CP = reinterpret_cast<double2(*)[BS][BS]>(lds);                      // 4 x 16 x 16, over M
    double2 mv[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int e = tid + h * kRoundThreads, i = e >> 5, j = e & 31;
      mv[h] = Ain[(size_t)pair_index(r - 1, nb, pp, i) * npad + pair_index(r - 1, nb, pq, j)];
    }
    double2 ux[2], uy[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = tid + h * kRoundThreads, k = e >> 4, j = e & 15;
      ux[h] = Ucur[(size_t)pp * SB * SB + k * SB + op + j];
      uy[h] = Ucur[(size_t)pq * SB * SB + k * SB + oq + j];
    }
    const double2 att = Ain[(size_t)(P * BS + a) * npad + P * BS + b];
    const double2 abb = Ain[(size_t)(Q * BS + a) * npad + Q * BS + b];
    const double2 ftt = Scur[(size_t)pp * 512 + (op ? 256 : 0) + a * BS + b];
    const double2 fbb = Scur[(size_t)pq * 512 + (oq ? 256 : 0) + a * BS + b];
    const bool idp = idp_raw != 0, idq = idq_raw != 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = tid + h * kRoundThreads, k = e >> 4, j = e & 15;
      Ux[k][j] = idp ? make_double2(k == op + j ? 1.0 : 0.0, 0.0) : ux[h];
      Uy[k][j] = idq ? make_double2(k == oq + j ? 1.0 : 0.0, 0.0) : uy[h];
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int e = tid + h * kRoundThreads;
      M[e >> 5][e & 31] = mv[h];
    }
    stt = idp ? att : ftt;
    sbb = idq ? abb : fbb;
    __syncthreads();
    // On the matrix cores (lane (g, m) = (lane / 16, lane % 16) supplies
    // A[m][4c + g] and B[4c + g][m]; results hold rows g + 4v of column m).
    // L = M Uy: wave w forms row tile w & 1 over k-half w >> 1.
    const int wave = tid >> 6, lane = tid & 63, g = lane >> 4, m = lane & 15;
    auto mma = [](double x, double y, double4_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0); };
    {
      const int rt = wave & 1, kh = wave >> 1;
      double4_t lr = {0.0, 0.0, 0.0, 0.0}, li = lr;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int k = (kh * 4 + c) * 4 + g;
        const double2 av = M[rt * BS + m][k], bv = Uy[k][m];
        lr = mma(av.x, bv.x, lr);
        lr = mma(-av.y, bv.y, lr);
        li = mma(av.x, bv.y, li);
        li = mma(av.y, bv.x, li);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) LP[kh][rt * BS + g + 4 * v][m] = make_double2(lr[v], li[v]);
    }
    __syncthreads();
    {
      // C = Ux' (LP[0] + LP[1]): wave w takes k-steps 2w, 2w + 1; partial
      // tiles summed in wave order below
      double4_t cr = {0.0, 0.0, 0.0, 0.0}, ci = cr;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int k = (wave * 2 + c) * 4 + g;
        const double2 u = Ux[k][m], l = cadd(LP[0][k][m], LP[1][k][m]);
        cr = mma(u.x, l.x, cr);
        cr = mma(u.y, l.y, cr);
        ci = mma(u.x, l.y, ci);
        ci = mma(-u.y, l.x, ci);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) CP[wave][g + 4 * v][m] = make_double2(cr[v], ci[v]);
    }
    __syncthreads();
    stb = cadd(cadd(CP[0][a][b], CP[1][a][b]), cadd(CP[2][a][b], CP[3][a][b]));
    sbt = cconj(cadd(cadd(CP[0][b][a], CP[1][b][a]), cadd(CP[2][b][a], CP[3][b][a])));
    __syncthreads();  // the LDS is reused below
  }
  // Exchange buffers, double buffered by inner round parity (one barrier
  // per round: a round's writes go to the buffer the previous round's reads
  // did not use).  Per buffer: the Q parts of S, the Q parts of U (two rows
  // per thread) and the P-P diagonal entries.
  constexpr int kXB = 16 * 17 * 16;  // bytes of one 16 x 17 double2 array
  constexpr int kXSet = 5 * kXB + 16 * 8;
  auto xtb = [&](int p) { return reinterpret_cast<double2(*)[BS + 1]>(lds + p * kXSet); };
  auto xbt = [&](int p) { return reinterpret_cast<double2(*)[BS + 1]>(lds + p * kXSet + kXB); };
  auto xbb = [&](int p) { return reinterpret_cast<double2(*)[BS + 1]>(lds + p * kXSet + 2 * kXB); };
  auto xu = [&](int p, int h) { return reinterpret_cast<double2(*)[BS + 1]>(lds + p * kXSet + (3 + h) * kXB); };
  auto xd = [&](int p) { return reinterpret_cast<double*>(lds + p * kXSet + 5 * kXB); };
  double* d0a = reinterpret_cast<double*>(lds + 2 * kXSet);
  double* d0b = d0a + BS;
  double2* d0c = reinterpret_cast<double2*>(d0b + BS);
  int* flag = reinterpret_cast<int*>(d0c + BS);
  if (tid == 0) {
    flag[0] = 0;
    flag[1] = 0;
  }
  if (a == b) {
    d0a[a] = stt.x;
    d0b[a] = sbb.x;
    d0c[a] = stb;
  }
  __syncthreads();
  // rotation inputs of index b (diagonal 2x2 block of round 0)
  const double aa = d0a[a];
  double ab = d0a[b], bb = d0b[b];
  double2 cb = d0c[b];
  {
    // early exit when no cross entry is above the rotation thresholds
    const double v2 = stb.x * stb.x + stb.y * stb.y;
    if (v2 > fl * fl && v2 > tol * tol * fabs(aa * bb)) flag[0] = 1;
  }
  __syncthreads();
  if (flag[0] == 0) {
    if (tid == 0) idnext[pair] = 1;
    return;
  }
  // Thread (a, b) also holds U rows b and b + 16 at P a and Q s(a).
  double2 ut[2], ub[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    ut[h] = make_double2(b + BS * h == a ? 1.0 : 0.0, 0.0);
    ub[h] = make_double2(b + BS * h == BS + a ? 1.0 : 0.0, 0.0);
  }
  int nrot = 0;
  const int a1 = (a + 1) & 15, b1 = (b + 1) & 15;
  for (int k = 0; k < BS; ++k) {
    // Each lane forms rotation b (its column index) and takes rotation a
    // from the lane of its row group whose column index is a: every wave
    // holds all 16 columns, so no rotation is formed more than four times.
    Rot ra, rb;
    const bool did = make_rot_fast(ab, bb, cb, tol, fl, &rb);
    {
      const int src = (tid & 63 & ~15) | a;
      ra.cs = __shfl(rb.cs, src);
      ra.sn = __shfl(rb.sn, src);
      ra.e.x = __shfl(rb.e.x, src);
      ra.e.y = __shfl(rb.e.y, src);
    }
    if (a == b) nrot += did;
    rot2x2(ra, rb, stt, stb, sbt, sbb);
    if (a == b && did) {
      stb = sbt = make_double2(0.0, 0.0);
      stt.y = sbb.y = 0.0;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      // U <- U J for pair a: new P = cs uP - sn conj(e) uQ, new Q = sn uP + cs conj(e) uQ
      const double2 w = cmul(ub[h], cconj(ra.e));
      const double2 up = ut[h];
      ut[h] = cadd(csc(ra.cs, up), csc(-ra.sn, w));
      ub[h] = cadd(csc(ra.sn, up), csc(ra.cs, w));
    }
    if (k == BS - 1) break;
    const int pb = k & 1;
    xtb(pb)[a][b] = stb;
    xbt(pb)[a][b] = sbt;
    xbb(pb)[a][b] = sbb;
    xu(pb, 0)[a][b] = ub[0];
    xu(pb, 1)[a][b] = ub[1];
    if (a == b) xd(pb)[a] = stt.x;
    __syncthreads();
    // s advances by one: Q parts from thread row / column + 1
    stb = xtb(pb)[a][b1];
    sbt = xbt(pb)[a1][b];
    sbb = xbb(pb)[a1][b1];
    ub[0] = xu(pb, 0)[a1][b];
    ub[1] = xu(pb, 1)[a1][b];
    // diagonal block of index t after the shift: P-P entry unchanged,
    // P-Q entry from block (t, t + 1), Q-Q entry from block (t + 1, t + 1)
    ab = xd(pb)[b];
    cb = xtb(pb)[b][b1];
    bb = xbb(pb)[b1][b1].x;
  }
  // After inner round 15 the Q parts sit at s(x) = x + 15.
  if (nrot) atomicAdd(&flag[1], nrot);
  __syncthreads();
  const int tot = flag[1];
  if (tid == 0) idnext[pair] = tot == 0;
  if (tot == 0) return;
  double2* out = Unext + (size_t)pair * SB * SB;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = b + BS * h;
    out[i * SB + a] = ut[h];
    out[i * SB + BS + ((a + BS - 1) & 15)] = ub[h];
  }
  double2* sf = Snext + (size_t)pair * 512;
  sf[a * BS + b] = stt;
  sf[256 + ((a + BS - 1) & 15) * BS + ((b + BS - 1) & 15)] = sbb;
}

// Apply role: the block update of round r on the FP64 matrix cores.  One
// workgroup per unordered pair alpha <= beta of index pairs: Aout[ia, ib]
// = Ua' Ain[ia, ib] Ub and, for alpha < beta, its mirror Aout[ib, ia] =
// Aout[ia, ib]'; V[ia, ib] <- V[ia, ib] Ub and V[ib, ia] <- V[ib, ia] Ua in
// place.  Wave (ti, tj) owns the 16 x 16 tiles (ti, tj) of T = Ua' B
// (exchanged through LDS), of T Ub and of the V blocks.  Complex products
// are four real v_mfma_f64_16x16x4 per k-step of 4 (operand of lane (g, m)
// = (lane / 16, lane % 16): A[m][4c + g] and B[4c + g][m]; the result holds
// rows g + 4v of column m).  Operands come straight from global memory
// (identity for pairs that did not rotate, whose U was not written).  With
// `sums`, squared Frobenius norms of the off-diagonal part and of the
// whole of both blocks (indices < n).
__device__ void apply_role(const double2* Ain, double2* Aout, double2* V, int n, int npad, int nb, int npair, int r,
                           int task, const double2* Ubuf, const int* ident, double* sums, unsigned char* lds) {
  auto Ttr = reinterpret_cast<double(*)[SB + 2]>(lds);
  auto Tti = reinterpret_cast<double(*)[SB + 2]>(lds + SB * (SB + 2) * 8);
  double* red = reinterpret_cast<double*>(lds + 2 * SB * (SB + 2) * 8);
  int alpha = 0, rem = task;
  while (rem >= npair - alpha) {
    rem -= npair - alpha;
    ++alpha;
  }
  const int beta = alpha + rem;
  const bool ida = ident[alpha] != 0, idb = ident[beta] != 0;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, m = lane & 15;
  const double2* ua = Ubuf + (size_t)alpha * SB * SB;
  const double2* ub = Ubuf + (size_t)beta * SB * SB;
  auto uval = [&](const double2* u, bool id, int k, int j) {
    return id ? make_double2(k == j ? 1.0 : 0.0, 0.0) : u[k * SB + j];
  };
  auto mma = [](double x, double y, double4_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0); };
  const int ti = wave >> 1, tj = wave & 1;
  const int im = ti * BS + m, jm = tj * BS + m;
  {
    // T = Ua' B, B = Ain[ia, ib]: A operand conj(Ua[k][im]), B operand B[k][jm]
    const size_t col = (size_t)pair_index(r, nb, beta, jm);
    double2 av[8], bv[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int k = 4 * c + g;
      av[c] = uval(ua, ida, k, im);
      bv[c] = Ain[(size_t)pair_index(r, nb, alpha, k) * npad + col];
    }
    double4_t tr = {0.0, 0.0, 0.0, 0.0}, tm = tr;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      tr = mma(av[c].x, bv[c].x, tr);
      tr = mma(av[c].y, bv[c].y, tr);
      tm = mma(av[c].x, bv[c].y, tm);
      tm = mma(-av[c].y, bv[c].x, tm);
    }
    // stored k-major for the next product: Tt[k][i] = T[i][k]
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Ttr[jm][ti * BS + g + 4 * v] = tr[v];
      Tti[jm][ti * BS + g + 4 * v] = tm[v];
    }
  }
  // V tiles: the two waves of a tile row read the whole row stripe, so the
  // in-place results are stored only after the barrier below.
  auto vtile = [&](int pr, int pc, const double2* u, double4_t& orr, double4_t& oi) {
    const size_t row = (size_t)pair_index(r, nb, pr, im) * npad;
    double2 av[8], bv[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int k = 4 * c + g;
      av[c] = V[row + pair_index(r, nb, pc, k)];
      bv[c] = u[k * SB + jm];
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      orr = mma(av[c].x, bv[c].x, orr);
      orr = mma(-av[c].y, bv[c].y, orr);
      oi = mma(av[c].x, bv[c].y, oi);
      oi = mma(av[c].y, bv[c].x, oi);
    }
  };
  auto vstore = [&](int pr, int pc, const double4_t& orr, const double4_t& oi) {
    const int gc = pair_index(r, nb, pc, jm);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      V[(size_t)pair_index(r, nb, pr, ti * BS + g + 4 * v) * npad + gc] = make_double2(orr[v], oi[v]);
  };
  const bool v1 = !idb, v2 = alpha < beta && !ida;
  double4_t o1r = {0.0, 0.0, 0.0, 0.0}, o1i = o1r, o2r = o1r, o2i = o1r;
  if (v1) vtile(alpha, beta, ub, o1r, o1i);
  if (v2) vtile(beta, alpha, ua, o2r, o2i);
  __syncthreads();
  if (v1) vstore(alpha, beta, o1r, o1i);
  if (v2) vstore(beta, alpha, o2r, o2i);
  // O = T Ub: A operand T[im][k] = Tt[k][im], B operand Ub[k][jm]
  double4_t orr = {0.0, 0.0, 0.0, 0.0}, oi = orr;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int k = 4 * c + g;
    const double2 bb = uval(ub, idb, k, jm);
    const double ar = Ttr[k][im], ai = Tti[k][im];
    orr = mma(ar, bb.x, orr);
    orr = mma(-ai, bb.y, orr);
    oi = mma(ar, bb.y, oi);
    oi = mma(ai, bb.x, oi);
  }
  double off2 = 0.0, all2 = 0.0;
  const int gc = pair_index(r, nb, beta, jm);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int gr = pair_index(r, nb, alpha, ti * BS + g + 4 * v);
    const double2 o = make_double2(orr[v], oi[v]);
    Aout[(size_t)gr * npad + gc] = o;
    if (alpha < beta) Aout[(size_t)gc * npad + gr] = cconj(o);
    if (gr < n && gc < n) {
      const double e2 = o.x * o.x + o.y * o.y;
      all2 += e2;
      if (gr != gc) off2 += e2;
    }
  }
  if (sums) {
    const double w = alpha < beta ? 2.0 : 1.0;  // the mirror block
    off2 = warp_sum_d(off2 * w);
    all2 = warp_sum_d(all2 * w);
    if (lane == 0) {
      red[wave] = off2;
      red[4 + wave] = all2;
    }
    __syncthreads();
    if (tid == 0) {
      sums[2 * task] = (red[0] + red[1]) + (red[2] + red[3]);
      sums[2 * task + 1] = (red[4] + red[5]) + (red[6] + red[7]);
    }
  }
}

// One launch per round: workgroups [0, npr) solve round r_apply + 1's
// subproblems (npr = npair, or 0 for the last round of a sweep), the rest
// apply round r_apply's rotations (Ain -> Aout, V in place).  Both roles
// read only what earlier launches wrote, so they need no ordering between
// them.
__global__ __launch_bounds__(kRoundThreads) void round_kernel(
    const double2* Ain, double2* Aout, double2* V, int n, int npad, int nb, int npair, int r_apply, int npr,
    const double2* Ucur, const int* idcur, const double2* Scur, double2* Unext, int* idnext, double2* Snext,
    double tol, const double* floor_dev, double* sums) {
  __shared__ __align__(16) unsigned char lds[kRoundLds];
  if ((int)blockIdx.x < npr)
    pair_role(Ain, npad, nb, r_apply + 1, blockIdx.x, Ucur, idcur, Scur, Unext, idnext, Snext, tol, *floor_dev, lds);
  else
    apply_role(Ain, Aout, V, n, npad, nb, npair, r_apply, blockIdx.x - npr, Ucur, idcur, sums, lds);
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

// C = op(X) Y for npad x npad complex matrices (op = conj-transpose when
// ct) on the FP64 matrix cores: one wave per 16 x 16 tile of C, four real
// v_mfma_f64_16x16x4 per k-step of 4 (lane (g, m) supplies op(X)[i0 + m]
// [k + g] and Y[k + g][j0 + m]), operands read from global memory eight
// k-steps ahead.
__global__ __launch_bounds__(256) void zgemm_kernel(const double2* X, const double2* Y, double2* C, int npad,
                                                    int ct) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, m = lane & 15;
  const int i0 = blockIdx.y * 32 + (wave >> 1) * 16, j0 = blockIdx.x * 32 + (wave & 1) * 16;
  auto xval = [&](int k) {
    return ct ? cconj(X[(size_t)k * npad + i0 + m]) : X[(size_t)(i0 + m) * npad + k];
  };
  double4_t cr = {0.0, 0.0, 0.0, 0.0}, ci = cr;
  constexpr int U = 8;
  for (int k0 = 0; k0 < npad; k0 += 4 * U) {
    double2 av[U], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + 4 * u + g;
      const bool in = k < npad;
      av[u] = in ? xval(k) : make_double2(0.0, 0.0);
      bv[u] = in ? Y[(size_t)k * npad + j0 + m] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].x, bv[u].x, cr, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[u].y, bv[u].y, cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].x, bv[u].y, ci, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].y, bv[u].x, ci, 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) C[(size_t)(i0 + g + 4 * v) * npad + j0 + m] = make_double2(cr[v], ci[v]);
}
// Ascending order of the n real eigenvalues (ties by index): perm[rank] = i.
__global__ __launch_bounds__(256) void rank_kernel(const double2* A, int n, int npad, int* perm, double* vals) {
  __shared__ double dgl[1024];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double li = i < n ? A[(size_t)i * npad + i].x : 0.0;
  int rk = 0;
  for (int j0 = 0; j0 < n; j0 += 1024) {
    const int cnt = min(1024, n - j0);
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += blockDim.x) dgl[j] = A[(size_t)(j0 + j) * npad + j0 + j].x;
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const double lj = dgl[j];
      rk += (lj < li) || (lj == li && j0 + j < i);
    }
  }
  if (i < n) {
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
  size_t A, A2, V, T, U, ident, S, part, perm, vals, sums, total;
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
  L.A2 = take(mat);
  L.V = take(mat);
  L.T = take(mat);
  L.U = take(2 * npair * SB * SB * sizeof(double2));
  L.ident = take(2 * npair * sizeof(int));
  L.S = take(2 * npair * 2 * BS * BS * sizeof(double2));
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
  const int np = npad_of(n), nb = np / BS, npair = nb / 2, nwg = npair * (npair + 1) / 2;
  const size_t mat = (size_t)np * np;
  char* base = reinterpret_cast<char*>(ws);
  double2* Abuf[2] = {reinterpret_cast<double2*>(base + L.A), reinterpret_cast<double2*>(base + L.A2)};
  double2* A = Abuf[0];
  double2* V = reinterpret_cast<double2*>(base + L.V);
  double2* T = reinterpret_cast<double2*>(base + L.T);
  // per-round outputs of the pair solves, double buffered by round parity
  double2* Ubuf[2] = {reinterpret_cast<double2*>(base + L.U),
                      reinterpret_cast<double2*>(base + L.U) + (size_t)npair * SB * SB};
  int* idbuf[2] = {reinterpret_cast<int*>(base + L.ident), reinterpret_cast<int*>(base + L.ident) + npair};
  double2* Sbuf[2] = {reinterpret_cast<double2*>(base + L.S),
                      reinterpret_cast<double2*>(base + L.S) + (size_t)npair * 2 * BS * BS};
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
  // Round r's pair outputs go to buffer (r + 2) % 2.  A sweep is the
  // opening round's pair solves, then nb - 1 launches that each apply round
  // r - 1 (A[cur] -> A[cur ^ 1]) while solving round r, then the last apply.
  auto par = [](int r) { return (r + 2) & 1; };
  int cur = 0;
  // Each sweep's convergence sums reach the host through pinned memory of
  // this host thread while the GPU already runs the next sweep's opening
  // round, which writes only the round buffers (no effect on A or V when
  // the host then stops).  The memory is coherent and mapped: sums_kernel
  // stores into it directly (a copy launch after it took about 12 us per
  // sweep), and the event's system-scope release makes the stores visible
  // to the host once the event has completed.
  static thread_local double* h_sums = nullptr;
  static thread_local double* h_sums_dev = nullptr;  // device address of h_sums
  if (!h_sums)
    HICU_HIP_TRY(hipHostMalloc((void**)&h_sums, 4 * sizeof(double),
                               hipHostMallocCoherent | hipHostMallocMapped | hipHostMallocPortable));
  if (!h_sums_dev) HICU_HIP_TRY(hipHostGetDevicePointer((void**)&h_sums_dev, h_sums, 0));
  HostWait done;
  HICU_HIP_TRY(done.init());
  auto opening = [&]() {
    // opening round: blocks (2 j, 2 j + 1) with all their index pairs
    hipLaunchKernelGGL(pair_eig_kernel, dim3(npair), dim3(1024), 0, st, (const double2*)Abuf[cur], np, nb, -1,
                       tol_inner, (const double*)dfloor, Ubuf[par(-1)], idbuf[par(-1)], Sbuf[par(-1)]);
  };
  opening();
  for (;;) {
    for (int r = 0; r <= nb - 1; ++r) {
      const bool last = r == nb - 1;  // apply only
      const int npr = last ? 0 : npair;
      hipLaunchKernelGGL(round_kernel, dim3(npr + nwg), dim3(kRoundThreads), 0, st, (const double2*)Abuf[cur],
                         Abuf[cur ^ 1], V, n, np, nb, npair, r - 1, npr, (const double2*)Ubuf[par(r - 1)],
                         (const int*)idbuf[par(r - 1)], (const double2*)Sbuf[par(r - 1)], Ubuf[par(r)],
                         idbuf[par(r)], Sbuf[par(r)], tol_inner, (const double*)dfloor, last ? part : nullptr);
      cur ^= 1;
    }
    hipLaunchKernelGGL(sums_kernel, dim3(1), dim3(256), 0, st, (const double*)part, nwg, h_sums_dev);
    HICU_HIP_TRY(hipGetLastError());
    ++sweeps;
    HICU_HIP_TRY(hipEventRecord(done.e, st));
    opening();  // the next sweep's, on the chance that this one has not converged
    HICU_HIP_TRY(hipGetLastError());
    HICU_HIP_TRY(done.poll());
    sums[0] = h_sums[0];
    sums[1] = h_sums[1];
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
  A = Abuf[cur];
  hipLaunchKernelGGL(rank_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, (const double2*)A, n, np,
                     perm, vals);
  hipLaunchKernelGGL(gather_kernel, dim3(n), dim3(256), 0, st, (const double2*)V, n, np, n - rank,
                     (const int*)perm, reinterpret_cast<float2*>(Q), reinterpret_cast<double2*>(Vout));
  if (evals)
    hipLaunchKernelGGL(copy_vals_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, (const double*)vals,
                       evals, n);
  HICU_HIP_TRY(hipGetLastError());
  return status;
}

}  // namespace hicu
