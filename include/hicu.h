/*
 * hicu.h — C ABI of the MI355X HICU hot-path library (libhicu.so).
 *
 * HICU (Zhao, Potter, Ahmad: "High-dimensional fast convolutional framework
 * for calibrationless MRI") recovers unobserved k-space by alternating
 * between a nullspace (annihilating-filter) estimate and gradient steps on
 * the residual energy of the multi-coil valid convolution (Algorithm 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named *_dev are DEVICE pointers on the current HIP device;
 *   pointers named *_host are host pointers.  The caller allocates and owns
 *   every buffer; the library never frees or retains caller buffers.
 * - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *   Calls enqueue work and return, except where "synchronous" is stated.
 *   Scalar results (J, ||g||^2, eta) are written to device memory so that a
 *   loop of calls needs no host synchronisation.
 * - Complex data are interleaved (re, im) pairs: complex64 = 2 x float,
 *   complex128 = 2 x double.
 * - k-space x is stored [d0][d1][d2][c] (coil c fastest, "coil-interleaved");
 *   spatial axes with index 0 slowest.  Fewer than three spatial axes are
 *   expressed with leading extents of 1 (see hicu_geom).
 * - Arguments are validated before any launch; on error nothing is written
 *   and a negative hicu_status is returned.  HIP runtime failures map to
 *   HICU_ERR_HIP.  No exception crosses this boundary.
 */
#ifndef HICU_H
#define HICU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HICU_OK = 0,
  HICU_CONVERGED = 1,          /* informational: gradient is exactly zero */
  HICU_ERR_ARG = -1,           /* NULL pointer / bad enum / bad count */
  HICU_ERR_SHAPE = -2,         /* inconsistent geometry, region smaller than kernel */
  HICU_ERR_RANK = -3,          /* rank outside [0, n) or p outside its range */
  HICU_ERR_NONFINITE = -4,     /* a NaN/Inf reached a scalar the loop depends on */
  HICU_ERR_HIP = -5,           /* HIP runtime error */
  HICU_ERR_WORKSPACE = -6,     /* workspace missing or too small */
  HICU_ERR_UNSUPPORTED = -7,   /* valid request the library does not implement */
  HICU_ERR_NOCONV = -8         /* eigensolver hit its sweep limit */
} hicu_status;

/* Operand precision of the im2col contractions (forward convolution,
 * adjoint convolution, line-search convolution).  Accumulation is always
 * FP32; scalar reductions finish in FP64.
 *   HICU_FP32   FP32 operands on the FP32 matrix cores.
 *   HICU_BF16   BF16 operands (round-to-nearest-even), one MFMA per tile.
 *   HICU_FP16   FP16 operands (round-to-nearest-even).  Each contraction's
 *               input is first multiplied by a power of two 2^(14 - e),
 *               e = ceil(log2 max|input|), so the largest magnitude lies
 *               in [2^13, 2^14] (no overflow at 65504; the scale is exact
 *               and undone in FP32 after accumulation).  Not available in
 *               the batched entry points.
 *   HICU_BF16X3 each FP32 operand split into hi + lo BF16 parts, three
 *               MFMAs (hi*hi + hi*lo + lo*hi) per tile: ~16-bit mantissa. */
typedef enum { HICU_FP32 = 0, HICU_BF16 = 1, HICU_BF16X3 = 2, HICU_FP16 = 3 } hicu_prec;

/* Problem geometry (THEORY section: k-space array, kernel mask, region S).
 * ndim      1..3 spatial axes.  Entries of dims/kdims/lo/hi beyond ndim are
 *           ignored; axes are right-aligned internally, i.e. a 2-D problem
 *           [d0][d1][c] is handled as [1][d0][d1][c].
 * nchan     coils Nc >= 1; the kernel always spans all coils, so one valid
 *           convolution also sums over coils.
 * dims      array extents.
 * kdims     rectangular kernel box; n = prod(kdims) * nchan taps.
 * lo, hi    region S = [lo, hi) per axis on which H is built (the centre-out
 *           box or the whole array); requires 0 <= lo, hi <= dims,
 *           hi - lo >= kdims.  Valid outputs u satisfy lo <= u <= hi - K.
 * wrap      bit a set: the convolution along axis a (of the ndim given) is
 *           circular instead of valid (METHODS, Study II: circular along
 *           time for 2-D+t).  That axis's region must be the whole axis
 *           (lo = 0, hi = dims, kdims <= dims); every position is an output
 *           and patch indices wrap modulo dims.  0 = all valid.  The batched
 *           entry points and the autotuner refuse circular axes
 *           (HICU_ERR_UNSUPPORTED), and so does hicu_gram's direct route
 *           (route 0 or more than 32 coils).
 * kmask     HOST pointer to prod(kdims) bytes (row-major over the kernel box,
 *           0 / nonzero) giving the support of the annihilating kernels
 *           (THEORY: the {0,1} kernel mask; DISCUSSION: circular or
 *           spherical supports), or NULL for the whole box.  The taps are
 *           the offsets with nonzero mask in lexicographic order, coil
 *           fastest, so n = (number of nonzero entries) * nchan; F, G and Q
 *           use that tap order.  The contractions run on the bounding box
 *           with zero weights outside the mask; the Gram is the box Gram
 *           restricted to the mask's taps.  Boxes of up to 512 offsets; the
 *           batched entry points and the autotuner refuse masks
 *           (HICU_ERR_UNSUPPORTED).  Read during the call only. */
typedef struct {
  int32_t ndim;
  int32_t nchan;
  int64_t dims[3];
  int32_t kdims[3];
  int64_t lo[3];
  int64_t hi[3];
  int32_t wrap;
  const uint8_t* kmask;
} hicu_geom;

/* Library version (major*10000 + minor*100 + patch). */
int32_t hicu_version(void);

/* Static description of a status code. */
const char* hicu_status_string(int32_t status);

/* Number of taps n = prod(kdims) * nchan, or a negative status. */
int64_t hicu_num_taps(const hicu_geom* geom);

/* Number of valid outputs s of region S, or a negative status. */
int64_t hicu_num_outputs(const hicu_geom* geom);

/* ------------------------------------------------------------------------
 * Gram matrix G = H_S(x)' H_S(x)   (DISCUSSION: Gram-matrix route to the
 * nullspace; THEORY: H(x) is the multi-level Hankel matrix of x on S).
 *   G[(k,c),(k',c')] = sum_{u valid} conj(x[u+k, c]) * x[u+k', c']
 * Row/column index = (k0, k1, k2, c) lexicographic, coil fastest.
 * x_dev   complex64 array of the full geometry.
 * G_dev   complex128 n x n, row-major, both triangles written.
 * Products and accumulation are FP64 (x is read as FP32 and widened).
 * ws_dev  device workspace of at least hicu_gram_workspace_bytes(geom).
 * ------------------------------------------------------------------------ */
size_t hicu_gram_workspace_bytes(const hicu_geom* geom);
int32_t hicu_gram(const hicu_geom* geom, const void* x_dev, void* G_dev,
                  void* ws_dev, size_t ws_bytes, void* stream);

/* Route of hicu_gram (process-wide; default 1).  Both give G to FP64
 * rounding from the same exact products:
 *   1  shift correlation: G[(k,c),(k+d,c')] depends on the tap pair only
 *      through the shift d and the window of summation points, so the
 *      region is cut into cells (single planes near both ends of each axis
 *      and one core segment) whose coil-by-coil correlation sums for every
 *      shift d >= 0 are formed once on the FP64 matrix cores and added per
 *      window: (2K-1)^D/2 shifts x Nc^2 coil pairs x |S| points of work
 *      instead of n^2 s / 2.  Up to 32 coils (more use route 0).
 *   0  direct products over the upper block triangle of the real Gram.
 * The workspace size covers both routes.  Returns HICU_OK, or
 * HICU_ERR_ARG for another value. */
int32_t hicu_set_gram_route(int32_t route);

/* ------------------------------------------------------------------------
 * Nullspace basis from the Gram (THEORY: J(x) of Eq. 1 equals
 * min ||H(x) Q||_F^2 over orthonormal Q with n - r columns; Algorithm 1,
 * nullspace update).  FP64 Hermitian eigendecomposition on the device by
 * block-Jacobi.
 * G_dev      complex128 n x n Hermitian (read only).
 * V0_dev     optional complex128 n x n unitary warm start (e.g. the previous
 *            call's eigenvectors), NULL for identity.
 * Q_dev      complex64 n x (n - r) row-major: eigenvectors of the n - r
 *            smallest eigenvalues in ascending order, each scaled by a unit
 *            phase so that the sum of its entries is real and >= 0.
 * evals_dev  optional double[n], all eigenvalues ascending.
 * V_dev      optional complex128 n x n, all eigenvectors (columns, same
 *            order and phase rule as Q), usable as the next warm start.
 * sweeps_host optional: number of Jacobi sweeps used.
 * Synchronous on `stream` (the convergence test reads two sums per sweep,
 * through 32 bytes of pinned host memory that the first call on a host
 * thread allocates and keeps until the process ends).
 * Returns HICU_ERR_NOCONV if 40 sweeps neither bring the off-diagonal
 * Frobenius norm below 1e-13 of the whole nor reach the rounding floor
 * (below 1e-10 and no longer halving per sweep); outputs are still written.
 * ------------------------------------------------------------------------ */
size_t hicu_nullspace_workspace_bytes(int32_t n);
int32_t hicu_nullspace(int32_t n, int32_t rank, const void* G_dev, const void* V0_dev,
                       void* Q_dev, double* evals_dev, void* V_dev, int32_t* sweeps_host,
                       void* ws_dev, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Nullspace basis by randomized SVD and Householder completion (THEORY:
 * first numerical technique; Algorithm 1, rSVD and Householder steps; cost
 * model).  The paper's own route: H_S(x) and its adjoint are applied to a
 * sketch, and neither the Hankel matrix nor its Gram is formed.
 *   1. Omega^(outer): n x l complex Gaussian test matrix (as hicu_sketch);
 *   2. Y = H_S(x) Omega by the FP32 forward contraction (s x l kept whole);
 *   3. W = H_S(x)' Y and M = Y'Y in one FP64 pass over the region
 *      (fixed-order sums, so the result is deterministic);
 *   4. V = the `rank` principal right singular vectors of B = U' H_S(x) with
 *      U an orthonormal basis of range(Y), from the eigendecompositions of M
 *      and of B B' (eigendirections of M below 1e-10 of its largest, the
 *      rounding floor of the FP32 sketch, are dropped);
 *   5. Q = the trailing n - rank columns of H_1 ... H_r, the Householder
 *      reflections of V's QR: H_j = I - 2 w w' with w the unit vector along
 *      a - alpha e_j, a the j-th column of the partly reduced V from row j
 *      down, alpha = -exp(i arg a_0) ||a|| (exp(i arg 0) = 1).
 * ell        sketch columns l with rank <= l <= n; 0 = ceil(3 rank / 2)
 *            capped at n (the paper's 3r/2 applications of H and H').
 * seed, outer, stream_id  counter words of the sketch draw.
 * Q_dev      complex64 n x (n - rank), row-major (no phase rule: the
 *            reflections fix the basis).
 * sv_dev     optional double[l]: singular values of B, largest first.
 * sweeps_host optional: Jacobi sweeps of the eigensolve of B B'.
 * Memory: the s x l complex64 sketch Y dominates (the paper's 1.5 r s).
 * rank = 0 writes the identity.  Kernel masks and circular axes are
 * supported; n above 2048 returns HICU_ERR_UNSUPPORTED.  Synchronous on
 * `stream`.  Returns HICU_ERR_NOCONV if the eigensolve of B B' hit its
 * sweep limit (outputs are still written).
 * ------------------------------------------------------------------------ */
size_t hicu_nullspace_rsvd_workspace_bytes(const hicu_geom* geom, int32_t rank, int32_t ell);
int32_t hicu_nullspace_rsvd(const hicu_geom* geom, const void* x_dev, int32_t rank, int32_t ell, uint64_t seed,
                            uint32_t outer, uint32_t stream_id, void* Q_dev, double* sv_dev, int32_t* sweeps_host,
                            void* ws_dev, size_t ws_bytes, void* stream);

/* The sketch Omega alone: complex64 n x ell row-major; element e has real
 * part z[2e] and imaginary part z[2e + 1], z the unit normals of the Philox
 * stream (seed, outer, 2^32 - 1, stream_id) mapped as in hicu_jl_compress
 * (no 1/sqrt(p) scale).  The inner word 2^32 - 1 is never a gradient-step
 * index, so no JL draw repeats a sketch draw. */
int32_t hicu_sketch(int32_t n, int32_t ell, uint64_t seed, uint32_t outer, uint32_t stream_id, void* Om_dev,
                    void* stream);

/* ------------------------------------------------------------------------
 * JL compression F = Q P   (THEORY: second numerical technique; Algorithm 1,
 * JL step).  P is real (nq x p), i.i.d. N(0, 1/p), drawn on the device from
 * Philox4x32-10 with key (seed lo, seed hi) and counter
 * (element/4, outer, inner, stream_id); each 4-word block gives four normals
 * by Box-Muller with u = (w + 1/2) 2^-32.
 * Q_dev  complex64 n x nq row-major; F_dev complex64 n x p row-major.
 * P_dev  optional double nq x p output of the drawn matrix (for checking).
 * ------------------------------------------------------------------------ */
int32_t hicu_jl_compress(int32_t n, int32_t nq, int32_t p, const void* Q_dev,
                         uint64_t seed, uint32_t outer, uint32_t inner, uint32_t stream_id,
                         void* F_dev, double* P_dev, void* stream);

/* ------------------------------------------------------------------------
 * Objective and gradient (THEORY: Eq. 2 with hard data matching; Algorithm 1
 * gradient step).  With Y = H_S(x) F:
 *   J      = ||Y||_F^2
 *   g      = 2 (1 - M) o H_S'(Y F^H)      (= 2 dJ/d conj(x), zero at observed
 *                                          locations and outside S)
 *   gnorm2 = ||g||^2
 * x_dev     complex64 full array.
 * mask_dev  uint8 [d0][d1][d2], 1 = observed (broadcast over coils); NULL =
 *           nothing observed.
 * F_dev     complex64 n x p row-major (filters in columns).
 * J_dev, g_dev, gnorm2_dev  outputs; any may be NULL (g_dev NULL skips the
 *           adjoint).  J_dev/gnorm2_dev are single doubles.
 * ws_dev    at least hicu_workspace_bytes(geom, p, prec) bytes.
 * When s x p complex values of Y exceed the filter-group budget (16 GiB by
 * default), the filters are processed in groups (a multiple of 64 filters
 * each): Y of one group lives in the workspace and the adjoint of each group
 * is added into g.  J and g are the same sums taken in another order.  On
 * the BF16 path with tiles of several planes (volumes), a grouped Y is
 * stored as BF16 (4 bytes per complex value, so groups hold twice the
 * filters): the adjoint rounds Y to BF16 anyway, so g is unchanged.
 * ------------------------------------------------------------------------ */
size_t hicu_workspace_bytes(const hicu_geom* geom, int32_t p, int32_t prec);

/* Set the byte budget of Y above which the gradient groups its filters
 * (process-wide; 0 restores the 16 GiB default).  Workspace sizes queried
 * before a change may be too small after it (calls then return
 * HICU_ERR_WORKSPACE).  Returns HICU_OK. */
int32_t hicu_set_filter_group_budget(size_t bytes);

/* Filters per group that hicu_objective_grad uses for this geometry, p and
 * prec under the current budget (*filters = p when Y fits at once), and
 * whether that Y is the compact BF16 residual (*compact = 1; compact may be
 * NULL).  Host pointers.  Returns HICU_ERR_ARG / HICU_ERR_SHAPE for bad
 * arguments, as hicu_objective_grad would. */
int32_t hicu_filter_group(const hicu_geom* geom, int32_t p, int32_t prec, int32_t* filters, int32_t* compact);
int32_t hicu_objective_grad(const hicu_geom* geom, const void* x_dev, const uint8_t* mask_dev,
                            const void* F_dev, int32_t p, int32_t prec, double* J_dev,
                            void* g_dev, double* gnorm2_dev, void* ws_dev, size_t ws_bytes,
                            void* stream);

/* ------------------------------------------------------------------------
 * Exact line search (THEORY: third numerical technique; Algorithm 1 ELS
 * step).  Z = H_S(g) F;  eta = gnorm2 / (2 ||Z||_F^2), eta = 0 when Z = 0.
 * gnorm2_dev  device double from hicu_objective_grad.
 * eta_dev     device double output.
 * ------------------------------------------------------------------------ */
int32_t hicu_line_search(const hicu_geom* geom, const void* g_dev, const double* gnorm2_dev,
                         const void* F_dev, int32_t p, int32_t prec, double* eta_dev,
                         void* ws_dev, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * hicu_line_search without a workspace argument, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and result as
 * hicu_line_search; the workspace is a fixed device array inside the library
 * (hicu_line_search_noalloc_max_bytes() = 64 MiB per GPU, held until the
 * process ends), looked up once per device on the first call with that
 * device current.  The call allocates nothing.  Problems whose line-search
 * workspace (hicu_workspace_bytes without the residual Y) exceeds the
 * scratch return HICU_ERR_WORKSPACE with nothing written.  Calls on one GPU
 * share its scratch: calls that overlap in time on one GPU (other streams,
 * other host threads) race and must be serialised by the caller.
 * Profiling (hicu_profile_begin) does not time these calls.
 * ------------------------------------------------------------------------ */
size_t hicu_line_search_noalloc_max_bytes(void);
int32_t hicu_line_search_noalloc(const hicu_geom* geom, const void* g_dev, const double* gnorm2_dev,
                                 const void* F_dev, int32_t p, int32_t prec, double* eta_dev,
                                 void* stream);

/* ------------------------------------------------------------------------
 * Time-averaged initialisation (METHODS, Study II: the initial k-space is
 * the time average; a phase-encoding point sampled in no frame is zero).
 * Along `axis` (0-based among the ndim axes of geom, the time frames), every
 * unobserved sample takes the mean of the observed samples of the same
 * location and coil over all frames; locations observed in no frame stay
 * zero; observed samples are copied unchanged.  Means are summed in FP64
 * over increasing frame index and rounded to FP32 once.
 * x0_dev    complex64 zero-filled observations; mask_dev uint8 [d0][d1][d2]
 *           (required); x_out_dev complex64, may alias x0_dev.
 * Only geom's dims and nchan are used (region, kernel and wrap are ignored
 * but must form a valid geometry).
 * ------------------------------------------------------------------------ */
int32_t hicu_time_average_init(const hicu_geom* geom, int32_t axis, const void* x0_dev,
                               const uint8_t* mask_dev, void* x_out_dev, void* stream);

/* x <- x - eta g over the whole array (Algorithm 1 update); eta read from
 * device memory.  Observed entries stay bit-identical because g is zero
 * there.  A zero or non-finite eta leaves x untouched (hicu_line_search
 * returns eta = 0 when any scalar it reads is non-finite, so a poisoned
 * gradient never reaches x). */
int32_t hicu_update(const hicu_geom* geom, void* x_dev, const void* g_dev,
                    const double* eta_dev, void* stream);

/* ------------------------------------------------------------------------
 * Full reconstruction, Algorithm 1 (nullspace by the Gram eigendecomposition or
 * by randomized SVD, see hicu_params.route).
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t rank;             /* r: 0 <= r < n */
  int32_t p;                /* filters per step: 0 = whole nullspace (no JL), else JL to p */
  int32_t n_outer;          /* I */
  int32_t start_outer;      /* resume: first outer iteration to run (0-based) */
  const int32_t* steps;     /* host int32[n_outer]: G^(i) gradient steps */
  const int64_t* regions;   /* host int64[n_outer][6]: lo[0..2] then hi[0..2], the first ndim
                               entries of each used as in hicu_geom; NULL = whole array */
  uint64_t seed;            /* JL seed */
  int32_t prec;             /* hicu_prec of the contractions */
  int32_t refine_steps;     /* the last refine_steps gradient steps of the run use refine_prec */
  int32_t warm_start;       /* 1: start each eigensolve from the previous eigenvectors (route 0) */
  int32_t route;            /* nullspace update: 0 = eigendecomposition of the Gram (DISCUSSION),
                               1 = randomized SVD + Householder (THEORY), as hicu_nullspace_rsvd
                               with the sketch of outer iteration i drawn for (seed, i, stream 0) */
  int32_t sketch;           /* route 1: sketch columns l (0 = ceil(3 rank / 2)) */
  int32_t refine_prec;      /* hicu_prec of the refine steps: HICU_FP32 (0, the default) or
                               HICU_BF16X3 (split operands on the BF16 matrix cores) */
} hicu_params;

/* One record per gradient step, filled when trace_host != NULL
 * (host array of sum(steps[start_outer..]) records). */
typedef struct {
  int32_t outer, inner, prec, sweeps;
  double J, gnorm2, eta;
} hicu_trace;

/* With p = 0 the iterates depend on the nullspace only through Q Q', so
 * the eigensolver stops resolving rotations below 1e-13 of the largest Gram
 * diagonal entry (its own rounding level); with JL (p > 0) the individual
 * eigenvectors matter and are resolved as in hicu_nullspace.
 * x0_dev    complex64 zero-filled observations (full array).
 * mask_dev  uint8 observed mask (may be NULL).
 * x_out_dev complex64 result; may alias x0_dev.
 * ws_dev    device workspace of at least hicu_solve_workspace_bytes(geom,
 *           params) bytes (0 for invalid arguments); the call allocates no
 *           device memory (the eigensolver's 32-byte pinned host slot, see
 *           hicu_nullspace, is allocated on a thread's first call only).
 * Synchronous (it reads the step scalars once per outer iteration).
 * Non-finite values: an x0 holding NaN/Inf is rejected with
 * HICU_ERR_NONFINITE before anything is written.  If a J, ||g||^2 or eta
 * turns non-finite during the run, the steps from there on are zero steps,
 * the run stops after that outer iteration with HICU_ERR_NONFINITE, and
 * x_out holds the last finite iterate; trace records of steps not run have
 * outer = inner = prec = -1. */
size_t hicu_solve_workspace_bytes(const hicu_geom* geom, const hicu_params* params);
int32_t hicu_solve(const hicu_geom* geom, const void* x0_dev, const uint8_t* mask_dev,
                   const hicu_params* params, void* x_out_dev, hicu_trace* trace_host,
                   void* ws_dev, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Batched gradient steps (Algorithm 1 gradient, ELS and update steps for many
 * independent problems: slices or frames of uneven size and coil count).
 * Every contraction of the step runs as ONE persistent launch over the work
 * list of all (problem, tile) items; reductions are per problem in a fixed
 * order, so each problem's result is bitwise the same as with the
 * single-problem calls on the same tile shape.
 *
 * hicu_batch_item:
 *   geom     geometry and region S of the problem
 *   x        complex64 k-space, DEVICE, updated in place by every step
 *   mask     uint8 observed mask or NULL
 *   Q        complex64 n x nq nullspace basis (row-major), DEVICE
 *   nq       columns of Q; p filters per step: p == nq uses Q itself, p < nq
 *            draws P^(i,j) (JL, as hicu_jl_compress with stream_id = the
 *            item's index) from the batch counter (i, j)
 *   seed     JL seed
 *   scalars  DEVICE double[3]: J, ||g||^2 and eta of the latest step
 *
 * hicu_batch_create   validates and plans (host only); *ws_bytes receives the
 *                     device workspace size.  The handle is host memory owned
 *                     by the library until hicu_batch_destroy.
 * hicu_batch_bind     binds a workspace (caller-owned, >= ws_bytes), uploads
 *                     the work tables and sets the JL counter to (0, 0);
 *                     synchronous.
 * hicu_batch_set_counter  sets the JL counter (i, j) with a kernel (no memset),
 *                     so it can sit in a captured graph.
 * hicu_batch_step     enqueues one step for every problem (kernel launches
 *                     only; capturable); the JL inner index j is incremented
 *                     on the device at the end of the step.
 * hicu_batch_graph_create  captures `steps` consecutive steps into one HIP
 *                     graph on `stream` (non-NULL); hicu_batch_graph_launch
 *                     replays it.
 * hicu_batch_info     info[6]: count, forward work items, adjoint work items,
 *                     forward tile code, adjoint tile code, workspace bytes.
 * ------------------------------------------------------------------------ */
typedef struct {
  hicu_geom geom;
  void* x;
  const uint8_t* mask;
  const void* Q;
  int32_t nq;
  int32_t p;
  uint64_t seed;
  double* scalars;
} hicu_batch_item;

typedef struct hicu_batch_s hicu_batch;

int32_t hicu_batch_create(const hicu_batch_item* items, int32_t count, int32_t prec, hicu_batch** out,
                          size_t* ws_bytes);
int32_t hicu_batch_bind(hicu_batch* batch, void* ws_dev, size_t ws_bytes, void* stream);
int32_t hicu_batch_set_counter(hicu_batch* batch, uint32_t outer, uint32_t inner, void* stream);
int32_t hicu_batch_step(hicu_batch* batch, void* stream);
int32_t hicu_batch_graph_create(hicu_batch* batch, int32_t steps, void* stream);
int32_t hicu_batch_graph_launch(hicu_batch* batch, void* stream);
int32_t hicu_batch_info(const hicu_batch* batch, int64_t* info);
void hicu_batch_destroy(hicu_batch* batch);

/* ------------------------------------------------------------------------
 * Tile-shape autotuner.  hicu_autotune times every valid tile shape of the
 * forward and adjoint contractions on the given problem (x, F, p, prec) with
 * HIP events and stores the fastest in a process-wide cache that every later
 * plan with the same (contraction, precision, kernel box, coils, filters,
 * size class) uses.  choice (optional, int32[4]): forward shape id and
 * channel chunk, adjoint shape id and channel chunk.  Synchronous.  Shapes
 * are timed on one filter group of the gradient (all p filters when Y = H(x)F
 * fits the filter-group budget), so the workspace never exceeds a step's.
 * hicu_autotune_batched does the same over the shapes that have persistent
 * batched kernels and stores the result for the batched runtime:
 * hicu_batch_create takes the batched choice stored for the class of its
 * largest problem (most n p s), else its fixed rule.  Neither tunes FP16
 * for the batch (the batched path runs no FP16).  hicu_tune_save /
 * hicu_tune_load write / read the cache as text (load returns the number
 * of entries read or a negative status); hicu_tune_clear empties it.
 * ------------------------------------------------------------------------ */
size_t hicu_autotune_workspace_bytes(const hicu_geom* geom, int32_t p, int32_t prec);
int32_t hicu_autotune(const hicu_geom* geom, const void* x_dev, const void* F_dev, int32_t p, int32_t prec,
                      void* ws_dev, size_t ws_bytes, int32_t* choice, void* stream);
int32_t hicu_autotune_batched(const hicu_geom* geom, const void* x_dev, const void* F_dev, int32_t p,
                              int32_t prec, void* ws_dev, size_t ws_bytes, int32_t* choice, void* stream);
int32_t hicu_tune_save(const char* path);
int32_t hicu_tune_load(const char* path);
int32_t hicu_tune_clear(void);
/* Pin the tile shape of one contraction (role 0 forward/line search, role 1
 * adjoint; roles 2 and 3 the same for the batched runtime, shapes with
 * batched kernels only; tile = shape id < hicu_tile_count(), a packing
 * shape (D > 1) only for role 1; chunk_c = adjoint channel chunk) for
 * problems of this geometry, filter count and precision. */
int32_t hicu_tune_put(const hicu_geom* geom, int32_t p, int32_t prec, int32_t role, int32_t tile,
                      int32_t chunk_c);

/* The contraction kernels' tile shapes.  Shape `tile` covers T0 x 16 x
 * (T2 * D) output positions and 16 * WC * FN launch columns per workgroup
 * of four waves (wave grid (4 / (WC KS)) x WC x KS; each wave an FM x FN
 * grid of 16 x 16 MFMA tiles); D > 1 packs D neighbouring outputs along
 * the last axis into the columns; KS > 1 has KS waves share each
 * fragment, taking every KS-th k-step, their sums added through LDS.
 * cfg receives int32[6] = {T0, T2, WC, FN, D, KS}. */
int32_t hicu_tile_count(void);
int32_t hicu_tile_info(int32_t tile, int32_t* cfg);

/* ------------------------------------------------------------------------
 * Per-kernel timing (tracing aid, not part of the method).  Between
 * hicu_profile_begin() and hicu_profile_end() every library launch is
 * bracketed by HIP events recorded on its own stream.  hicu_profile_end()
 * waits for those events and returns one record per kernel class (up to
 * max_stats; *n_stats receives the number of classes).  flops/bytes are the
 * algorithmic work summed over the class's launches (the convolutions count
 * 8 n p s real flops each: one complex multiply-add per tap, filter and
 * output; the Gram 4 s n^2, the count of a Hermitian product H'H).
 * Process-wide; not meant for concurrent use from several threads.
 * hicu_profile_begin_major() times only the contractions, the Gram, the
 * eigensolver, the rSVD and JL steps and the batched launches: the per-step
 * scalar and layout kernels (reductions, line-search step, update, weight
 * layouts, scaling) go untimed, which keeps the events' own cost (a few us
 * per record) out of a timed run.
 * ------------------------------------------------------------------------ */
typedef struct {
  char name[24];
  int64_t launches;
  double total_ms, min_ms, max_ms;
  double flops, bytes;
} hicu_kernel_stat;

int32_t hicu_profile_begin(void);
int32_t hicu_profile_begin_major(void);
int32_t hicu_profile_end(hicu_kernel_stat* stats, int32_t max_stats, int32_t* n_stats);

#ifdef __cplusplus
}
#endif

#endif /* HICU_H */
