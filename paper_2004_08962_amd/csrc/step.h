// One gradient step of the method for one problem: forward convolution with
// the objective, adjoint convolution with hard data matching, line-search
// convolution (THEORY section; Algorithm 1, gradient and ELS steps).
#pragma once

#include "common.h"
#include "conv.h"

namespace hicu {

constexpr size_t kAlign = 256;
inline size_t al(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
inline char* at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

inline bool valid_prec(int p) { return p == P_F32 || p == P_BF16 || p == P_BF16X3 || p == P_F16; }
inline size_t esize(int prec) { return prec == P_F32 ? 4 : 2; }

// Bytes of H_S(x)F kept in device memory at once: above this the gradient
// runs over groups of filters (forward into Y, adjoint accumulated into g),
// since Y = s x p complex values (200 MB per filter for a 256x320x320 volume
// with a 5x5x5 kernel) does not fit for hundreds of filters.
constexpr size_t kYBudget = size_t(16) << 30;

// Filters per group for s valid outputs, p filters and `bytes` per stored
// residual value: all of them when Y fits the budget, else the largest
// multiple of 64 that does (at least 64).
int filter_group(int64_t s, int p, size_t bytes = 8);
// Replace the budget (0 restores kYBudget); process-wide.
void set_y_budget(size_t bytes);

// Workspace layout of one step (offsets from the workspace base).
struct StepPlan {
  WeightShape wf, wa;
  ConvPlan cf, ca;      // forward over all filters (also the line search), adjoint
  int pc;               // filters per group of the gradient
  int ybw;              // > 0: Y stored as BF16 in blocks of ybw filters (BF16 path, grouped); 0: complex64
  size_t off_Y, off_Bf, off_Bflo, off_Ba, off_Balo, off_pf, off_pa, off_pz, off_sc, off_pmax, total;
  int64_t nf_blocks, na_blocks;
};

int32_t plan_forward(const Geo& g, int p, int prec, WeightShape* w, ConvPlan* c);
int32_t plan_adjoint(const Geo& g, int p, int prec, WeightShape* w, ConvPlan* c);
int32_t make_step_plan(const Geo& g, int p, int prec, bool need_adj, StepPlan* sp);
const char* conv_tag(int kind, int prec);
int64_t region_points(const Geo& g);
bool full_region(const Geo& g);

// Fill the pointer/stride/epilogue fields of sp.cf.a for H_S(in) F.
void fill_forward_args(const Geo& g, const void* in, StepPlan& sp, void* ws, float* out, double* partial);

// Fill sp.ca.a-style arguments for 2 (1 - M) o H_S'(Y F^H) written to gout.
void fill_adjoint_args(const Geo& g, const void* Y, int p, const void* B, const void* Blo, void* gout,
                       const uint8_t* mask, double* partial, ConvArgs& a);

// Which filter-weight layouts objective_grad_impl builds from F before its
// contractions.  A caller that ran it on the same F, precision, geometry and
// workspace earlier may skip the rebuild (the weights are left in place).
constexpr int kPrepForward = 1, kPrepAdjoint = 2, kPrepAll = 3;

int32_t objective_grad_impl(const Geo& g, const void* x, const uint8_t* mask, const void* F, int p, int prec,
                            double* J, void* gout, double* gn2, void* ws, size_t ws_bytes, hipStream_t st,
                            int prep = kPrepAll);
// grad_weights: reuse the forward weights objective_grad_impl left in the
// same workspace for the same F, precision and geometry (no rebuild).
int32_t line_search_impl(const Geo& g, const void* gv, const double* gn2, const void* F, int p, int prec,
                         double* eta, void* ws, size_t ws_bytes, hipStream_t st, bool grad_weights = false);
size_t step_workspace(const Geo& g, int p, int prec);
// Y = H_S(x) F stored whole as s x p complex64 (point-major, filter fastest),
// for any precision but FP16.
size_t forward_store_workspace(const Geo& g, int p, int prec);
int32_t forward_store_impl(const Geo& g, const void* x, const void* F, int p, int prec, void* Y, void* ws,
                           size_t ws_bytes, hipStream_t st);

}  // namespace hicu
