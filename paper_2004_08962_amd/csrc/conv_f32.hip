// Instantiations of the contraction kernels for one precision (split from
// the host code so the precisions compile in parallel).
#include "conv_impl.h"

namespace hicu {

template int32_t launch_prec_impl<P_F32>(const ConvPlan& p, bool pipe, hipStream_t st);
template int32_t launch_batch_prec_impl<P_F32>(const BatchConvLaunch& b, hipStream_t st);

}  // namespace hicu
