// Stencil kernels of order 6 (see pn_launch.h).
#include "pn_launch.h"

namespace pn {
template hipError_t launch_order<6>(int, bool, bool, const StencilArgs&, hipStream_t);
}  // namespace pn
