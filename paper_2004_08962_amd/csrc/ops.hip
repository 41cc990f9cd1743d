// Small device operations of the gradient loop: JL compression of the
// nullspace, the exact-line-search step size, the update, zero fill.
#include <algorithm>

#include "ops.h"
#include "philox.h"

namespace hicu {

// JL: block (j, b) forms column j of F = Q P for rows [64 b, 64 b + 64).
__global__ __launch_bounds__(256) void jl_kernel(const float2* Q, int n, int nq, int p, uint64_t seed,
                                                 uint32_t outer, uint32_t inner, uint32_t sid, float2* F,
                                                 double* Pout) {
  extern __shared__ double pcol[];
  jl_column_rows(Q, n, nq, p, blockIdx.x, blockIdx.y * kJlRows, seed, outer, inner, sid, pcol, F, Pout);
}

int32_t launch_jl(const float2* Q, int n, int nq, int p, uint64_t seed, uint32_t outer, uint32_t inner,
                  uint32_t sid, float2* F, double* Pout, hipStream_t st) {
  const size_t lds = (size_t)nq * sizeof(double);
  if (lds > 65536) return HICU_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(jl_kernel, dim3(p, (unsigned)cdiv(n, kJlRows)), dim3(256), lds, st, Q, n, nq, p, seed, outer,
                     inner, sid, F, Pout);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

// Sketch of the randomized SVD: Omega (n x l complex64, row-major); element
// e takes normals 2e (real part) and 2e + 1 (imaginary part) of the stream
// (seed, outer, 2^32 - 1, sid) -- the inner counter word 2^32 - 1 is never a
// gradient-step index, so the sketch shares no draw with the JL matrices.
__global__ __launch_bounds__(256) void sketch_kernel(int64_t count, uint64_t seed, uint32_t outer, uint32_t sid,
                                                     float2* Om) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const double re = philox_normal(2 * e, seed, outer, 0xFFFFFFFFu, sid);
  const double im = philox_normal(2 * e + 1, seed, outer, 0xFFFFFFFFu, sid);
  Om[e] = make_float2((float)re, (float)im);
}

int32_t launch_sketch(int n, int ell, uint64_t seed, uint32_t outer, uint32_t sid, float2* Om, hipStream_t st) {
  const int64_t count = (int64_t)n * ell;
  if (count <= 0) return HICU_OK;
  hipLaunchKernelGGL(sketch_kernel, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, st, count, seed, outer, sid, Om);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

// eta = gnorm2 / (2 sum(part)), 0 when the sum is 0 or anything is non-finite.
__global__ __launch_bounds__(1024) void eta_kernel(const double* part, int64_t count, const double* gnorm2,
                                                   double* eta) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += blockDim.x) s += part[i];
  const double zz = block_sum_d(s, red);
  if (threadIdx.x == 0) {
    const double gn = *gnorm2;
    double e = 0.0;
    if (zz > 0.0 && isfinite(zz) && isfinite(gn)) e = gn / (2.0 * zz);
    if (!isfinite(e)) e = 0.0;
    *eta = e;
  }
}

int32_t launch_eta(const double* part, int64_t count, const double* gnorm2, double* eta, hipStream_t st) {
  hipLaunchKernelGGL(eta_kernel, dim3(1), dim3(1024), 0, st, part, count, gnorm2, eta);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

// x <- x - eta g, evaluated in FP64 and rounded once.  A zero or non-finite
// eta leaves x untouched (the line search returns 0 for a zero gradient and
// for any non-finite scalar, so a poisoned gradient never reaches x).
__global__ void update_kernel(float2* x, const float2* g, const double* eta, int64_t count) {
  const double e = *eta;
  if (!(e != 0.0) || !isfinite(e)) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const float2 gv = g[i];
    float2 xv = x[i];
    xv.x = (float)((double)xv.x - e * (double)gv.x);
    xv.y = (float)((double)xv.y - e * (double)gv.y);
    x[i] = xv;
  }
}

int32_t launch_update(float2* x, const float2* g, const double* eta, int64_t count, hipStream_t st) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(count, 256), 16384));
  hipLaunchKernelGGL(update_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, g, eta, count);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

// Kernel mask: filters over the mask's taps (n rows) spread to the whole
// kernel box (nbox rows, zero rows outside the mask), p columns.
__global__ __launch_bounds__(256) void kmask_scatter_kernel(const float2* F, KMaskBits bits, int nc, int nbox, int p,
                                                            float2* Fbox) {
  const int64_t total = (int64_t)nbox * p;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(e / p), j = (int)(e % p);
    const int t = kmask_tap_of(bits.w, row / nc);
    Fbox[e] = t < 0 ? make_float2(0.f, 0.f) : F[((size_t)t * nc + row % nc) * p + j];
  }
}

int32_t launch_kmask_scatter(const Geo& g, const float2* F, int p, float2* Fbox, hipStream_t st) {
  KMaskBits kb;
  for (int w = 0; w < 8; ++w) kb.w[w] = g.kbits[w];
  const int64_t tot = (int64_t)g.nbox * p;
  hipLaunchKernelGGL(kmask_scatter_kernel, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(tot, 256), 16384))),
                     dim3(256), 0, st, F, kb, g.nc, g.nbox, p, Fbox);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

// Time-averaged initialisation (METHODS, Study II): along axis t, each
// (location, coil) column gets the mean of its observed samples at the
// unobserved ones; a column observed in no frame stays zero.  One thread per
// column; the points of a column are p = (o * nt + t) * inner + i.  Sums in
// FP64 in increasing t, one rounding to FP32.  Each thread reads and writes
// only its own column, so out may alias x0.
__global__ __launch_bounds__(256) void time_average_kernel(const float2* x0, const uint8_t* mask, float2* out,
                                                           int64_t outer, int64_t nt, int64_t inner, int nc) {
  const int64_t cols = outer * inner * nc;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cols; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % nc);
    const int64_t i = (e / nc) % inner, o = e / ((int64_t)nc * inner);
    double sr = 0.0, si = 0.0;
    int64_t cnt = 0;
    for (int64_t t = 0; t < nt; ++t) {
      const int64_t p = (o * nt + t) * inner + i;
      if (mask[p]) {
        const float2 v = x0[p * nc + c];
        sr += (double)v.x;
        si += (double)v.y;
        ++cnt;
      }
    }
    const float2 avg = cnt ? make_float2((float)(sr / (double)cnt), (float)(si / (double)cnt)) : make_float2(0.f, 0.f);
    for (int64_t t = 0; t < nt; ++t) {
      const int64_t p = (o * nt + t) * inner + i;
      out[p * nc + c] = mask[p] ? x0[p * nc + c] : avg;
    }
  }
}

int32_t launch_time_average(const float2* x0, const uint8_t* mask, float2* out, const int64_t d[3], int axis,
                            int nc, hipStream_t st) {
  int64_t outer = 1, inner = 1;
  for (int a = 0; a < axis; ++a) outer *= d[a];
  for (int a = axis + 1; a < 3; ++a) inner *= d[a];
  const int64_t cols = outer * inner * nc;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(cols, 256), 16384));
  hipLaunchKernelGGL(time_average_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x0, mask, out, outer, d[axis],
                     inner, nc);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

// Number of non-finite floats among v[0..count) added into *out (grid-stride,
// one atomic per block).
__global__ __launch_bounds__(256) void nonfinite_kernel(const float* v, int64_t count, unsigned long long* out) {
  __shared__ unsigned int red[4];
  unsigned int c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    c += isfinite(v[i]) ? 0u : 1u;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int t = red[0] + red[1] + red[2] + red[3];
    if (t) atomicAdd(out, (unsigned long long)t);
  }
}

__global__ void clear_u64_kernel(unsigned long long* p) { *p = 0ull; }

int32_t launch_count_nonfinite(const float* v, int64_t count, unsigned long long* out, hipStream_t st) {
  hipLaunchKernelGGL(clear_u64_kernel, dim3(1), dim3(1), 0, st, out);
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(count, 256), 4096));
  hipLaunchKernelGGL(nonfinite_kernel, dim3((unsigned)blocks), dim3(256), 0, st, v, count, out);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

__global__ void zero_kernel(float4_t* p, int64_t n4) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = float4_t{0.f, 0.f, 0.f, 0.f};
}

__global__ void zero_tail_kernel(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

// Zero-fill with a kernel (graph-capture friendly, no memset nodes).
int32_t launch_zero(void* ptr, size_t bytes, hipStream_t st) {
  if (bytes % 4 != 0) return HICU_ERR_ARG;
  const int64_t n4 = (int64_t)(bytes / 16);
  const int64_t tail = (int64_t)(bytes % 16) / 4;
  if (n4 > 0) {
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(n4, 256), 16384));
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, reinterpret_cast<float4_t*>(ptr), n4);
  }
  if (tail > 0)
    hipLaunchKernelGGL(zero_tail_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<float*>(ptr) + n4 * 4, tail);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

__global__ __launch_bounds__(256) void absmax_kernel(const float* v, int64_t count, float* part) {
  __shared__ float red[4];
  float m = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(v[i]));
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

int32_t launch_absmax(const float* v, int64_t count, float* part, hipStream_t st) {
  hipLaunchKernelGGL(absmax_kernel, dim3(kAbsmaxBlocks), dim3(256), 0, st, v, count, part);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

__global__ __launch_bounds__(256) void scale_kernel(const float* part, int64_t count, float* scale) {
  __shared__ float red[4];
  float m = 0.f;
  for (int64_t i = threadIdx.x; i < count; i += blockDim.x) m = fmaxf(m, part[i]);
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    float s = 1.f;
    if (m > 0.f && m < INFINITY) {
      int e;
      const float f = frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
      const int c = f > 0.5f ? e : e - 1;  // ceil(log2 m)
      s = ldexpf(1.f, max(-126, min(126, 14 - c)));
    }
    *scale = s;
  }
}

int32_t launch_scale(const float* part, int64_t count, float* scale, hipStream_t st) {
  hipLaunchKernelGGL(scale_kernel, dim3(1), dim3(256), 0, st, part, count, scale);
  HICU_HIP_TRY(hipGetLastError());
  return HICU_OK;
}

}  // namespace hicu
