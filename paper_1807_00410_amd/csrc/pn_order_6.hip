// Stencil kernels of order 6 (see pn_launch.h and pn_stencil_lds.h).
#include "pn_launch.h"

namespace pn {
template hipError_t launch_order<6>(int, bool, bool, const StencilArgs&, hipStream_t);
template hipError_t launch_lds_order<6>(int, bool, const StencilArgs&, hipStream_t);
template hipError_t lds_prepare<6>(size_t);
template hipError_t launch_batch_order<6>(int, bool, const BatchLaunch&, hipStream_t);
}  // namespace pn
