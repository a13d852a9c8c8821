// Stencil kernels of order 3 (see pn_launch.h).
#include "pn_launch.h"

namespace pn {
template hipError_t launch_order<3>(int, bool, bool, const StencilArgs&, hipStream_t);
}  // namespace pn
