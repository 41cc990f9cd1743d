// Randomized-SVD nullspace route (THEORY, first numerical technique;
// Algorithm 1, rSVD and Householder steps).
//
//  1. Sketch: Omega (n x l complex, N(0, 1) parts from Philox) and
//     Y = H_S(x) Omega by the forward contraction (FP32 operands and sums).
//  2. One pass over the region on the FP64 matrix cores forms
//     [H_S(x) | Y]' Y, i.e. W = H_S(x)' Y (the adjoint correlation applied
//     to the l sketch columns) and M = Y'Y, per range of positions; a second
//     kernel sums the ranges in a fixed order.
//  3. With M = Z D Z', U = Y Z D^-1/2 is an orthonormal basis of range(Y),
//     so B' = H_S(x)' U = W Z D^-1/2 without forming U.  Directions of M
//     below 1e-10 of its largest eigenvalue are dropped: they lie under the
//     rounding floor of the FP32 sketch.
//  4. C = B B' = E L E' (FP64 Jacobi); V = B' E_r L_r^-1/2 holds the r
//     principal right singular vectors of B, largest first.
//  5. Householder QR of V: reflector j is H_j = I - 2 w w' with w the unit
//     vector along a - alpha e_j, a the j-th column of the partly reduced V
//     from row j down and alpha = -exp(i arg a_0) ||a||, formed a panel of
//     up to 8 reflectors per launch.  The trailing n - r columns of
//     H_1 ... H_r are Q.
// Right singular vectors of U'H do not depend on which orthonormal basis U
// of range(Y) is used, so steps 3-4 give the V of a QR-based rSVD.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "eig.h"
#include "ops.h"
#include "prof.h"
#include "rsvd.h"
#include "step.h"

namespace hicu {

namespace {

constexpr int kProjAhead = 8;     // positions (steps of 4) fetched ahead
constexpr double kDropRel = 1e-10;  // relative floor on the eigenvalues of M

struct ProjArgs {
  const float* x;     // complex64 array viewed as floats
  const float* Y;     // s x l complex64 viewed as floats
  int64_t d1, d2;     // array extents of axes 1, 2
  int nc, n, ell;
  int K1, K2;         // kernel box extents of axes 1, 2
  int kmasked;
  uint64_t kbits[8];
  int64_t lo[3];
  int64_t per[3];     // extent of a circular axis, 0 otherwise
  int64_t m1, m2;     // valid extents of axes 1, 2
  int64_t s;
  int nra, ncb;       // real rows 2 (n + l), real columns 2 l
  int ntc, ntiles;    // 64-wide column tiles, tiles in all
  int64_t qper;       // positions per range (multiple of 4)
  int ngroups;
  double* part;       // [ngroups][ntiles][64][64]
};

__device__ __forceinline__ int64_t proj_remap(int64_t w, int64_t W) {
  const int64_t per = W / 8, rem = W % 8;
  const int64_t xcd = w % 8, idx = w / 8;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// Operand row of the real product: a tap of the patch (kind 0: tap offsets
// and float within the tap's coils), a float of the sketch row (kind 1), or
// padding (kind 2).
struct RowSrc {
  int kind;
  int k0, k1, k2, el;
  int col;
};

__device__ __forceinline__ RowSrc row_source(const ProjArgs& a, int e) {
  RowSrc r{2, 0, 0, 0, 0, 0};
  if (e < 2 * a.n) {
    const int t = e / (2 * a.nc);
    const int f = a.kmasked ? kmask_offset_of(a.kbits, t) : t;
    r.kind = 0;
    r.k2 = f % a.K2;
    r.k1 = (f / a.K2) % a.K1;
    r.k0 = f / (a.K2 * a.K1);
    r.el = e % (2 * a.nc);
  } else if (e < a.nra) {
    r.kind = 1;
    r.col = e - 2 * a.n;
  }
  return r;
}

__device__ __forceinline__ int64_t wrapped(int64_t i, int64_t per) { return (per && i >= per) ? i - per : i; }

// One 64 x 64 tile of [A_x | Y]^T Y (real embedding) over one position
// range; four waves of 32 x 32, each 2 x 2 MFMA tiles of 16 x 16.
__global__ __launch_bounds__(256) void proj_kernel(ProjArgs a) {
  const int64_t lin = proj_remap(blockIdx.x, (int64_t)a.ntiles * a.ngroups);
  const int tile = (int)(lin % a.ntiles), grp = (int)(lin / a.ntiles);
  const int I = tile / a.ntc, J = tile % a.ntc;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, m = lane & 15;
  const int wr = wave >> 1, wc = wave & 1;

  RowSrc ra[2];
  int cb[2];
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    ra[f] = row_source(a, I * 64 + wr * 32 + f * 16 + m);
    const int eb = J * 64 + wc * 32 + f * 16 + m;
    cb[f] = eb < a.ncb ? eb : -1;
  }

  double4_t acc[2][2];
#pragma unroll
  for (int f = 0; f < 2; ++f)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[f][j] = double4_t{0.0, 0.0, 0.0, 0.0};

  const int64_t q_begin = (int64_t)grp * a.qper;
  const int64_t q_end = std::min<int64_t>(a.s, q_begin + a.qper);
  const int64_t two_nc = 2 * a.nc, two_l = 2 * a.ell;
  // Lane group g walks positions q_begin + g, + 4, ...; (u0, u1, u2) follow q.
  int64_t q = q_begin + g;
  int64_t u2 = q % a.m2, u1 = (q / a.m2) % a.m1, u0 = q / (a.m2 * a.m1);
  // Without circular axes the operand of row f sits at a fixed offset from
  // the point's base in x (a tap) or in Y (a sketch column): the bases
  // advance with the point and no index is wrapped or recomputed per step.
  const bool wrap_any = a.per[0] != 0 || a.per[1] != 0 || a.per[2] != 0;
  const float* src[2];
  int64_t aoff[2];
  bool ax_[2], on_[2];
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    ax_[f] = ra[f].kind == 0;
    on_[f] = ra[f].kind != 2;
    src[f] = ax_[f] ? a.x : a.Y;
    aoff[f] = ax_[f] ? (((int64_t)ra[f].k0 * a.d1 + ra[f].k1) * a.d2 + ra[f].k2) * two_nc + ra[f].el
                     : (int64_t)ra[f].col;
  }
  auto xbase_of = [&]() { return (((a.lo[0] + u0) * a.d1 + (a.lo[1] + u1)) * a.d2 + (a.lo[2] + u2)) * two_nc; };
  int64_t xbase = xbase_of(), ybase = q * two_l;
  auto run = [&](auto wrap_tag) {
    constexpr bool WRAP = decltype(wrap_tag)::value;
    // Loads carry no select: lanes that are off read element 0 and the
    // masks are applied where the values are used (a select right after
    // a load makes the compiler wait for it where it is issued).
    auto fetch = [&](float (&av)[2], float (&bv)[2]) {
      const bool ok = q < q_end;
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const bool on = ok && on_[f];
        if constexpr (!WRAP) {
          av[f] = src[f][on ? (ax_[f] ? xbase : ybase) + aoff[f] : 0];
        } else {
          // both indices formed without branches (a branch here cost a
          // wait on the ring's loads)
          const int64_t i0 = wrapped(a.lo[0] + u0 + ra[f].k0, a.per[0]);
          const int64_t i1 = wrapped(a.lo[1] + u1 + ra[f].k1, a.per[1]);
          const int64_t i2 = wrapped(a.lo[2] + u2 + ra[f].k2, a.per[2]);
          const int64_t xi = ((i0 * a.d1 + i1) * a.d2 + i2) * two_nc + ra[f].el;
          av[f] = src[f][on ? (ax_[f] ? xi : ybase + ra[f].col) : 0];
        }
        const bool onb = ok && cb[f] >= 0;
        bv[f] = a.Y[onb ? ybase + cb[f] : 0];
      }
      q += 4;
      ybase += 4 * two_l;
      u2 += 4;
      if (u2 < a.m2) {
        xbase += 4 * two_nc;
      } else {
        while (u2 >= a.m2) {
          u2 -= a.m2;
          if (++u1 == a.m1) {
            u1 = 0;
            ++u0;
          }
        }
        xbase = xbase_of();
      }
    };
    constexpr int PF = kProjAhead;
    float av[PF][2], bv[PF][2];
#pragma unroll
    for (int r = 0; r < PF; ++r) fetch(av[r], bv[r]);
    // whole blocks of PF steps: steps past the range's end are masked
    for (int64_t q0 = q_begin; q0 < q_end; q0 += 4 * PF) {
#pragma unroll
      for (int r = 0; r < PF; ++r) {
        const bool ok = q0 + 4 * r + g < q_end;
        double ad[2], bd[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          ad[f] = (double)(av[r][f] * (ok && on_[f] ? 1.f : 0.f));
          bd[f] = (double)(bv[r][f] * (ok && cb[f] >= 0 ? 1.f : 0.f));
        }
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[f][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ad[f], bd[j], acc[f][j], 0, 0, 0);
        fetch(av[r], bv[r]);
      }
    }
  };
  if (wrap_any) run(std::true_type{});
  else run(std::false_type{});

  double* out = a.part + ((size_t)grp * a.ntiles + tile) * 4096;
#pragma unroll
  for (int f = 0; f < 2; ++f)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // v_mfma_f64_16x16x4: lane holds rows g, g + 4, g + 8, g + 12 of column m
        const int r = wr * 32 + f * 16 + g + 4 * i;
        const int c = wc * 32 + j * 16 + m;
        out[r * 64 + c] = acc[f][j][i];
      }
}

// Sum the ranges in order and form the complex entries O[a][j] =
// sum conj(Z[u][a]) Y[u][j]: rows a < n go to W (n x l), the rest to M
// (l x l, upper triangle mirrored so that M is exactly Hermitian).
__global__ __launch_bounds__(256) void proj_finalize_kernel(const double* part, int ngroups, int ntiles, int ntc,
                                                            int n, int ell, double2* W, double2* M) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)(n + ell) * ell) return;
  const int arow = (int)(idx / ell), j = (int)(idx % ell);
  if (arow >= n && arow - n > j) return;
  const int tile = (2 * arow / 64) * ntc + (2 * j / 64);
  const int lr = (2 * arow) % 64, lc = (2 * j) % 64;
  double rr = 0.0, ii = 0.0, ri = 0.0, ir = 0.0;
  for (int y = 0; y < ngroups; ++y) {
    const double* t = part + ((size_t)y * ntiles + tile) * 4096;
    rr += t[lr * 64 + lc];
    ii += t[(lr + 1) * 64 + lc + 1];
    ri += t[lr * 64 + lc + 1];
    ir += t[(lr + 1) * 64 + lc];
  }
  const double re = rr + ii;
  if (arow < n) {
    W[(size_t)arow * ell + j] = make_double2(re, ri - ir);
  } else {
    const int i = arow - n;
    const double im = i == j ? 0.0 : ri - ir;
    M[(size_t)i * ell + j] = make_double2(re, im);
    if (i != j) M[(size_t)j * ell + i] = make_double2(re, -im);
  }
}

// Dense complex FP64 products of the small matrices: C = A B with
// element (i, k) of A at A.p[i rs + k cs] (conjugated when A.conj).  With
// herm the result is Hermitian by construction: entries i <= j are computed
// and mirrored.
struct ZView {
  const double2* p;
  int64_t rs, cs;
  int conj;
};

__global__ __launch_bounds__(256) void zgemm_small_kernel(int M, int N, int K, ZView A, ZView B, double2* C,
                                                          int64_t crs, int64_t ccs, int herm) {
  __shared__ double2 sa[16][17], sb[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
  double cr = 0.0, ci = 0.0;
  for (int k0 = 0; k0 < K; k0 += 16) {
    {
      const int ai = blockIdx.y * 16 + ty, ak = k0 + tx;
      double2 v = make_double2(0.0, 0.0);
      if (ai < M && ak < K) v = A.p[ai * A.rs + ak * A.cs];
      if (A.conj) v.y = -v.y;
      sa[ty][tx] = v;
      const int bk = k0 + ty, bj = blockIdx.x * 16 + tx;
      double2 w = make_double2(0.0, 0.0);
      if (bk < K && bj < N) w = B.p[bk * B.rs + bj * B.cs];
      if (B.conj) w.y = -w.y;
      sb[ty][tx] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const double2 u = sa[ty][kk], v = sb[kk][tx];
      cr = fma(u.x, v.x, cr);
      cr = fma(-u.y, v.y, cr);
      ci = fma(u.x, v.y, ci);
      ci = fma(u.y, v.x, ci);
    }
    __syncthreads();
  }
  if (i >= M || j >= N) return;
  if (!herm) {
    C[i * crs + j * ccs] = make_double2(cr, ci);
  } else if (i <= j) {
    C[i * crs + j * ccs] = make_double2(cr, i == j ? 0.0 : ci);
    if (i != j) C[j * crs + i * ccs] = make_double2(cr, -ci);
  }
}

// Z D^-1/2 with the columns of eigenvalues below kDropRel of the largest set
// to zero (eigenvalues ascending, eigenvectors in columns, row-major l x l).
__global__ __launch_bounds__(256) void lowdin_kernel(double2* Z, const double* ev, int ell) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)ell * ell) return;
  const int j = (int)(idx % ell);
  const double top = ev[ell - 1], d = ev[j];
  const double s = (top > 0.0 && d > kDropRel * top) ? 1.0 / sqrt(d) : 0.0;
  const double2 z = Z[idx];
  Z[idx] = make_double2(z.x * s, z.y * s);
}

// The r largest eigenpairs of C, largest first: E_r L_r^-1/2 (l x r,
// row-major) and the singular values sqrt(L) of B, largest first.
__global__ __launch_bounds__(256) void top_kernel(const double2* E, const double* ev, int ell, int r, double2* Er,
                                                  double* sv) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sv && idx < ell) sv[idx] = sqrt(std::max(ev[ell - 1 - idx], 0.0));
  if (idx >= (int64_t)ell * r) return;
  const int i = (int)(idx / r), c = (int)(idx % r);
  const int src = ell - 1 - c;
  const double lam = ev[src];
  const double s = lam > 0.0 ? 1.0 / sqrt(lam) : 0.0;
  const double2 e = E[(size_t)i * ell + src];
  Er[idx] = make_double2(e.x * s, e.y * s);
}

// Householder QR of V (column-major, n x r) in panels of b columns.  Every
// block of a launch factors the panel (columns j0 .. j0 + b - 1 from row j0
// down) in LDS -- the same arithmetic in every block, so all hold identical
// reflectors -- then applies the b reflectors in order to its own trailing
// columns (one wave per column, the column in registers, NPL values per
// lane).  Block 0 stores the panel's unit reflector vectors in Wr.
// Reflector jj: w along a - alpha e_jj with alpha = -ph ||a||, ph the phase
// of a_0, so w_jj = ph (|a_0| + ||a||) and ||w||^2 = 2 ||a|| (||a|| + |a_0|).
template <int NPL>
__global__ __launch_bounds__(256) void hh_panel_kernel(double2* V, int n, int r, int j0, int b, double2* Wr) {
  extern __shared__ double2 pan[];  // [b][len]
  __shared__ double red[4];
  __shared__ double2 sh_w0;
  __shared__ double sh_inv;
  const int len = n - j0;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int e = tid; e < b * len; e += 256) {
    const int c = e / len, i = e - c * len;
    pan[e] = V[(size_t)(j0 + c) * n + j0 + i];
  }
  __syncthreads();
  for (int jj = 0; jj < b; ++jj) {
    double2* a = pan + (size_t)jj * len;
    double nr2 = 0.0;
    for (int i = jj + tid; i < len; i += 256) nr2 += a[i].x * a[i].x + a[i].y * a[i].y;
    nr2 = block_sum_d(nr2, red);
    if (tid == 0) {
      const double2 a0 = a[jj];
      const double norm = sqrt(nr2), mag0 = sqrt(a0.x * a0.x + a0.y * a0.y);
      const double2 ph = mag0 > 0.0 ? make_double2(a0.x / mag0, a0.y / mag0) : make_double2(1.0, 0.0);
      sh_w0 = make_double2(ph.x * (mag0 + norm), ph.y * (mag0 + norm));
      const double wn2 = 2.0 * norm * (norm + mag0);
      sh_inv = wn2 > 0.0 ? 1.0 / sqrt(wn2) : 0.0;
    }
    __syncthreads();
    const double inv = sh_inv;
    for (int i = jj + tid; i < len; i += 256) {
      const double2 v = i == jj ? sh_w0 : a[i];
      a[i] = make_double2(v.x * inv, v.y * inv);
    }
    __syncthreads();
    for (int c = jj + 1 + wave; c < b; c += 4) {
      double2* col = pan + (size_t)c * len;
      double dr = 0.0, di = 0.0;
      for (int i = jj + lane; i < len; i += 64) {
        const double2 w = a[i], v = col[i];
        dr += w.x * v.x + w.y * v.y;  // conj(w) v
        di += w.x * v.y - w.y * v.x;
      }
      dr = warp_sum_d(dr);
      di = warp_sum_d(di);
      for (int i = jj + lane; i < len; i += 64) {
        const double2 w = a[i], v = col[i];
        col[i] = make_double2(v.x - 2.0 * (w.x * dr - w.y * di), v.y - 2.0 * (w.x * di + w.y * dr));
      }
    }
    __syncthreads();
  }
  if (blockIdx.x == 0)
    for (int e = tid; e < b * len; e += 256) {
      const int c = e / len, i = e - c * len;
      if (i >= c) Wr[(size_t)(j0 + c) * n + j0 + i] = pan[e];
    }
  const int c = j0 + b + blockIdx.x * 4 + wave;
  if (c >= r) return;
  double2* col = V + (size_t)c * n + j0;
  double2 q[NPL];
#pragma unroll
  for (int t = 0; t < NPL; ++t) {
    const int i = t * 64 + lane;
    q[t] = i < len ? col[i] : make_double2(0.0, 0.0);
  }
  for (int jj = 0; jj < b; ++jj) {
    const double2* w = pan + (size_t)jj * len;
    double dr = 0.0, di = 0.0;
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int i = t * 64 + lane;
      if (i >= jj && i < len) {
        const double2 wv = w[i];
        dr += wv.x * q[t].x + wv.y * q[t].y;
        di += wv.x * q[t].y - wv.y * q[t].x;
      }
    }
    dr = warp_sum_d(dr);
    di = warp_sum_d(di);
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int i = t * 64 + lane;
      if (i >= jj && i < len) {
        const double2 wv = w[i];
        q[t].x -= 2.0 * (wv.x * dr - wv.y * di);
        q[t].y -= 2.0 * (wv.x * di + wv.y * dr);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NPL; ++t) {
    const int i = t * 64 + lane;
    if (i < len) col[i] = q[t];
  }
}

// Q = H_1 ... H_r [0; I]: one wave per column of Q holds it in registers
// (NPL values per lane) and applies H_r first, H_1 last.
template <int NPL>
__global__ __launch_bounds__(256) void hh_apply_kernel(const double2* Wr, int n, int r, float2* Q) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nq = n - r;
  const int c = blockIdx.x * 4 + wave;
  if (c >= nq) return;
  double2 q[NPL];
#pragma unroll
  for (int t = 0; t < NPL; ++t) q[t] = make_double2(t * 64 + lane == r + c ? 1.0 : 0.0, 0.0);
  for (int j = r - 1; j >= 0; --j) {
    const double2* w = Wr + (size_t)j * n;
    double dr = 0.0, di = 0.0;
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int i = t * 64 + lane;
      if (i >= j && i < n) {
        const double2 wv = w[i];
        dr += wv.x * q[t].x + wv.y * q[t].y;
        di += wv.x * q[t].y - wv.y * q[t].x;
      }
    }
    dr = warp_sum_d(dr);
    di = warp_sum_d(di);
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
      const int i = t * 64 + lane;
      if (i >= j && i < n) {
        const double2 wv = w[i];
        q[t].x -= 2.0 * (wv.x * dr - wv.y * di);
        q[t].y -= 2.0 * (wv.x * di + wv.y * dr);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NPL; ++t) {
    const int i = t * 64 + lane;
    if (i < n) Q[(size_t)i * nq + c] = make_float2((float)q[t].x, (float)q[t].y);
  }
}

__global__ void identity_kernel(float2* Q, int n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  Q[idx] = make_float2(idx / n == idx % n ? 1.f : 0.f, 0.f);
}

struct ProjLayout {
  int ntr, ntc, ntiles, ngroups;
  int64_t qper;
};

ProjLayout proj_layout(const Geo& g, int ell) {
  ProjLayout L;
  L.ntr = (int)cdiv(2 * (g.n + ell), 64);
  L.ntc = (int)cdiv(2 * ell, 64);
  L.ntiles = L.ntr * L.ntc;
  // Enough blocks to fill 256 CUs several times, at least 256 positions per range.
  int64_t groups = std::max<int64_t>(1, 4096 / L.ntiles);
  groups = std::min<int64_t>(groups, std::max<int64_t>(1, g.s / 256));
  L.qper = rup(cdiv(g.s, groups), 4);
  L.ngroups = (int)cdiv(g.s, L.qper);
  return L;
}

struct RsvdLayout {
  size_t om, y, fws, part, W, M, ZM, evM, eig, BH, C, ZC, evC, Er, V, Wr, total;
  size_t fws_bytes, eig_bytes;
};

RsvdLayout rsvd_layout(const Geo& g, int ell, int rank) {
  const ProjLayout P = proj_layout(g, ell);
  RsvdLayout L;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += al(b);
    return o;
  };
  const size_t n = (size_t)g.n, l = (size_t)ell, r = (size_t)rank;
  L.fws_bytes = forward_store_workspace(g, ell, P_F32);
  L.eig_bytes = eig_workspace(ell);
  L.om = take(n * l * sizeof(float2));
  L.y = take((size_t)g.s * l * sizeof(float2));
  L.fws = take(L.fws_bytes);
  L.part = take((size_t)P.ngroups * P.ntiles * 4096 * sizeof(double));
  L.W = take(n * l * sizeof(double2));
  L.M = take(l * l * sizeof(double2));
  L.ZM = take(l * l * sizeof(double2));
  L.evM = take(l * sizeof(double));
  L.eig = take(L.eig_bytes);
  L.BH = take(n * l * sizeof(double2));
  L.C = take(l * l * sizeof(double2));
  L.ZC = take(l * l * sizeof(double2));
  L.evC = take(l * sizeof(double));
  L.Er = take(l * r * sizeof(double2));
  L.V = take(n * r * sizeof(double2));
  L.Wr = take(n * r * sizeof(double2));
  L.total = L.fws_bytes ? off : 0;
  return L;
}

int32_t launch_zgemm(int M, int N, int K, ZView A, ZView B, double2* C, int64_t crs, int64_t ccs, bool herm,
                     hipStream_t st) {
  hipLaunchKernelGGL(zgemm_small_kernel, dim3((unsigned)cdiv(N, 16), (unsigned)cdiv(M, 16)), dim3(256), 0, st, M, N,
                     K, A, B, C, crs, ccs, herm ? 1 : 0);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

// Panel width: up to 8 columns of at most 120 KB of LDS.
int hh_panel_width(int n) { return (int)std::max<int64_t>(1, std::min<int64_t>(8, (120 << 10) / (16 * (int64_t)n))); }

template <int NPL>
int32_t launch_panels(double2* V, int n, int r, double2* Wr, hipStream_t st) {
  const int bw = hh_panel_width(n);
  for (int j0 = 0; j0 < r; j0 += bw) {
    const int b = std::min(bw, r - j0);
    const int cols = r - j0 - b;
    const size_t lds = (size_t)b * (n - j0) * sizeof(double2);
    hipLaunchKernelGGL(hh_panel_kernel<NPL>, dim3((unsigned)std::max<int64_t>(1, cdiv(cols, 4))), dim3(256), lds, st,
                       V, n, r, j0, b, Wr);
  }
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

template <int NPL>
int32_t launch_apply(const double2* Wr, int n, int r, float2* Q, hipStream_t st) {
  hipLaunchKernelGGL(hh_apply_kernel<NPL>, dim3((unsigned)cdiv(n - r, 4)), dim3(256), 0, st, Wr, n, r, Q);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

}  // namespace

size_t rsvd_workspace(const Geo& g, int rank, int ell) {
  if (rank == 0) return 0;
  return rsvd_layout(g, ell, rank).total;
}

int32_t run_rsvd(const Geo& g, const void* x, int rank, int ell, uint64_t seed, uint32_t outer, uint32_t sid,
                 float2* Q, double* sv, int32_t* sweeps, void* ws, size_t ws_bytes, hipStream_t st, bool basis) {
  const int n = g.n;
  if (n > kRsvdMaxN) return HICU_ERR_UNSUPPORTED;
  if (rank < 0 || rank >= n) return HICU_ERR_RANK;
  if (sweeps) *sweeps = 0;
  if (rank == 0) {
    hipLaunchKernelGGL(identity_kernel, dim3((unsigned)cdiv((int64_t)n * n, 256)), dim3(256), 0, st, Q, n);
    HICU_HIP_TRY(hipGetLastError());
    return HICU_OK;
  }
  if (ell < rank || ell > n) return HICU_ERR_ARG;
  const RsvdLayout L = rsvd_layout(g, ell, rank);
  if (L.total == 0) return HICU_ERR_UNSUPPORTED;
  if (!ws || ws_bytes < L.total) return HICU_ERR_WORKSPACE;
  float2* Om = reinterpret_cast<float2*>(at(ws, L.om));
  float2* Y = reinterpret_cast<float2*>(at(ws, L.y));
  double* part = reinterpret_cast<double*>(at(ws, L.part));
  double2* W = reinterpret_cast<double2*>(at(ws, L.W));
  double2* M = reinterpret_cast<double2*>(at(ws, L.M));
  double2* ZM = reinterpret_cast<double2*>(at(ws, L.ZM));
  double* evM = reinterpret_cast<double*>(at(ws, L.evM));
  double2* BH = reinterpret_cast<double2*>(at(ws, L.BH));
  double2* C = reinterpret_cast<double2*>(at(ws, L.C));
  double2* ZC = reinterpret_cast<double2*>(at(ws, L.ZC));
  double* evC = reinterpret_cast<double*>(at(ws, L.evC));
  double2* Er = reinterpret_cast<double2*>(at(ws, L.Er));
  double2* V = reinterpret_cast<double2*>(at(ws, L.V));
  double2* Wr = reinterpret_cast<double2*>(at(ws, L.Wr));

  // 1. sketch
  {
    ProfScope ps("rsvd_sketch", st);
    HICU_TRY(launch_sketch(n, ell, seed, outer, sid, Om, st));
  }
  HICU_TRY(forward_store_impl(g, x, Om, ell, P_F32, Y, at(ws, L.fws), L.fws_bytes, st));

  // 2. W = H' Y and M = Y'Y
  const ProjLayout P = proj_layout(g, ell);
  {
    ProjArgs a{};
    a.x = reinterpret_cast<const float*>(x);
    a.Y = reinterpret_cast<const float*>(Y);
    a.d1 = g.d[1];
    a.d2 = g.d[2];
    a.nc = g.nc;
    a.n = n;
    a.ell = ell;
    a.K1 = g.k[1];
    a.K2 = g.k[2];
    a.kmasked = g.kmasked;
    for (int w = 0; w < 8; ++w) a.kbits[w] = g.kbits[w];
    for (int i = 0; i < 3; ++i) {
      a.lo[i] = g.lo[i];
      a.per[i] = g.wrap[i] ? g.d[i] : 0;
    }
    a.m1 = g.m[1];
    a.m2 = g.m[2];
    a.s = g.s;
    a.nra = 2 * (n + ell);
    a.ncb = 2 * ell;
    a.ntc = P.ntc;
    a.ntiles = P.ntiles;
    a.qper = P.qper;
    a.ngroups = P.ngroups;
    a.part = part;
    ProfScope ps("rsvd_proj", st, 8.0 * (double)(n + ell) * ell * (double)g.s,
                 8.0 * (double)region_points(g) * g.nc + 8.0 * (double)g.s * ell);
    hipLaunchKernelGGL(proj_kernel, dim3((unsigned)((int64_t)P.ntiles * P.ngroups)), dim3(256), 0, st, a);
    HICU_HIP_TRY(hipGetLastError());
    const int64_t outs = (int64_t)(n + ell) * ell;
    hipLaunchKernelGGL(proj_finalize_kernel, dim3((unsigned)cdiv(outs, 256)), dim3(256), 0, st, (const double*)part,
                       P.ngroups, P.ntiles, P.ntc, n, ell, W, M);
    HICU_HIP_TRY(hipGetLastError());
  }

  // 3. B' = W Z D^-1/2 from the eigendecomposition of M
  int32_t sw = 0;
  {
    ProfScope ps("rsvd_eig", st);
    // any orthonormal basis of range(Y) serves, so M's eigenvectors need
    // only the eigensolver's projector accuracy
    const int32_t es = run_eig(ell, 0, M, nullptr, nullptr, evM, ZM, &sw, at(ws, L.eig), L.eig_bytes, st, true);
    if (es < 0 && es != HICU_ERR_NOCONV) return es;
  }
  hipLaunchKernelGGL(lowdin_kernel, dim3((unsigned)cdiv((int64_t)ell * ell, 256)), dim3(256), 0, st, ZM,
                     (const double*)evM, ell);
  HICU_HIP_TRY(hipGetLastError());
  HICU_TRY(launch_zgemm(n, ell, ell, ZView{W, ell, 1, 0}, ZView{ZM, ell, 1, 0}, BH, ell, 1, false, st));
  // 4. C = B B' and its r largest eigenpairs
  HICU_TRY(launch_zgemm(ell, ell, n, ZView{BH, 1, ell, 1}, ZView{BH, ell, 1, 0}, C, ell, 1, true, st));
  int32_t status = HICU_OK;
  {
    ProfScope ps("rsvd_eig", st);
    const int32_t es = run_eig(ell, 0, C, nullptr, nullptr, evC, ZC, &sw, at(ws, L.eig), L.eig_bytes, st, !basis);
    if (es < 0 && es != HICU_ERR_NOCONV) return es;
    if (es == HICU_ERR_NOCONV) status = es;
  }
  if (sweeps) *sweeps = sw;
  hipLaunchKernelGGL(top_kernel, dim3((unsigned)cdiv((int64_t)ell * std::max(rank, 1), 256)), dim3(256), 0, st,
                     (const double2*)ZC, (const double*)evC, ell, rank, Er, sv);
  HICU_HIP_TRY(hipGetLastError());
  // V (column-major n x r) = B' E_r L_r^-1/2
  HICU_TRY(launch_zgemm(n, rank, ell, ZView{BH, ell, 1, 0}, ZView{Er, rank, 1, 0}, V, 1, n, false, st));

  // 5. Householder completion
  {
    ProfScope ps("householder", st);
    HICU_TRY(launch_zero(Wr, (size_t)n * rank * sizeof(double2), st));
    const int npl = (int)cdiv(n, 64);
    if (npl <= 2) {
      HICU_TRY(launch_panels<2>(V, n, rank, Wr, st));
      HICU_TRY(launch_apply<2>(Wr, n, rank, Q, st));
    } else if (npl <= 4) {
      HICU_TRY(launch_panels<4>(V, n, rank, Wr, st));
      HICU_TRY(launch_apply<4>(Wr, n, rank, Q, st));
    } else if (npl <= 8) {
      HICU_TRY(launch_panels<8>(V, n, rank, Wr, st));
      HICU_TRY(launch_apply<8>(Wr, n, rank, Q, st));
    } else if (npl <= 16) {
      HICU_TRY(launch_panels<16>(V, n, rank, Wr, st));
      HICU_TRY(launch_apply<16>(Wr, n, rank, Q, st));
    } else if (npl <= 24) {
      HICU_TRY(launch_panels<24>(V, n, rank, Wr, st));
      HICU_TRY(launch_apply<24>(Wr, n, rank, Q, st));
    } else {
      HICU_TRY(launch_panels<32>(V, n, rank, Wr, st));
      HICU_TRY(launch_apply<32>(Wr, n, rank, Q, st));
    }
  }
  return status;
}

}  // namespace hicu
