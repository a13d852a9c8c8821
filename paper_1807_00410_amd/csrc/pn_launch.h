// Launch of the stencil kernel variants of one order.  Each order is
// instantiated in its own translation unit (pn_order_N.hip) so the library
// builds in parallel.
#pragma once
#include "pn_kernels.h"
#include "pn_stencil_lds.h"

namespace pn {

// Kernel flavours used by the library: (vector type, mode, output type).
enum Kind {
  K_F32_APPLY = 0,   // float  -> float  y = op(x)
  K_F32_TRANSR = 1,  // float  -> float  r' = r - alpha q, y = A^T r'
  K_F64_APPLY = 2,   // double -> double
  K_F64_TRANSR = 3,  // double -> double
  K_F64_RESID32 = 4, // double x, float Q -> float r = Q - A x
  K_F64_RESID64 = 5, // double x, float Q -> double r
  K_F32_SUPD = 6,    // float: s = s - alpha op(x) (CG on the normal equations)
  K_F32_APPLY_EQ = 7,// float: y = W A x (row-equilibrated CG)
  K_F32_EQS = 8,     // float: y = W x
  // float, even-parity Schur complement (one band parity of rows)
  K_F32_ODD_W = 9, K_F32_EVEN_S = 10, K_F32_EVEN_RHS = 11, K_F32_ODD_BACK = 12, K_F32_EVEN_JAC = 13,
  K_F32_EVEN_SR = 14
};

// modes whose kernels never reduce (instantiated without partial sums only)
constexpr bool mode_no_norm(int m) { return m == M_EVEN_RHS || m == M_ODD_BACK || m == M_EVEN_JAC; }

template <int N, typename T, int MODE, typename TO>
hipError_t launch_flavour(bool gen, bool norm, const StencilArgs& a, hipStream_t s) {
  dim3 grid(a.nblocks), block(kBlock);
  if constexpr (mode_no_norm(MODE)) {
    if (gen) hipLaunchKernelGGL((k_stencil<N, T, MODE, TO, true, false>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_stencil<N, T, MODE, TO, false, false>), grid, block, 0, s, a);
  } else if (MODE == M_APPLY && !norm) {
    if (gen) hipLaunchKernelGGL((k_stencil<N, T, MODE, TO, true, false>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_stencil<N, T, MODE, TO, false, false>), grid, block, 0, s, a);
  } else {
    if (gen) hipLaunchKernelGGL((k_stencil<N, T, MODE, TO, true, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_stencil<N, T, MODE, TO, false, true>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

template <int N>
hipError_t launch_order(int kind, bool gen, bool norm, const StencilArgs& a, hipStream_t s) {
  switch (kind) {
    case K_F32_APPLY: return launch_flavour<N, float, M_APPLY, float>(gen, norm, a, s);
    case K_F32_TRANSR: return launch_flavour<N, float, M_TRANSR, float>(gen, true, a, s);
    case K_F64_APPLY: return launch_flavour<N, double, M_APPLY, double>(gen, norm, a, s);
    case K_F64_TRANSR: return launch_flavour<N, double, M_TRANSR, double>(gen, true, a, s);
    case K_F64_RESID32: return launch_flavour<N, double, M_RESID, float>(gen, true, a, s);
    case K_F64_RESID64: return launch_flavour<N, double, M_RESID, double>(gen, true, a, s);
    case K_F32_SUPD: return launch_flavour<N, float, M_SUPD, float>(gen, true, a, s);
    case K_F32_APPLY_EQ: return launch_flavour<N, float, M_APPLY_EQ, float>(gen, true, a, s);
    case K_F32_EQS: return launch_flavour<N, float, M_EQS, float>(gen, true, a, s);
    case K_F32_ODD_W: return launch_flavour<N, float, M_ODD_W, float>(gen, true, a, s);
    case K_F32_EVEN_SR: return launch_flavour<N, float, M_EVEN_SR, float>(gen, true, a, s);
    case K_F32_EVEN_S: return launch_flavour<N, float, M_EVEN_S, float>(gen, true, a, s);
    case K_F32_EVEN_RHS: return launch_flavour<N, float, M_EVEN_RHS, float>(gen, false, a, s);
    case K_F32_ODD_BACK: return launch_flavour<N, float, M_ODD_BACK, float>(gen, false, a, s);
    case K_F32_EVEN_JAC: return launch_flavour<N, float, M_EVEN_JAC, float>(gen, false, a, s);
    default: return hipErrorInvalidValue;
  }
}

// Batched launch over the systems of one order (BatchLaunch.work); the
// Krylov kinds always reduce.
template <int N, typename T, int MODE, typename TO>
hipError_t launch_batch_flavour(bool gen, const BatchLaunch& bl, hipStream_t s) {
  dim3 grid(bl.nwork), block(kBlock);
  if (gen) hipLaunchKernelGGL((k_stencil_batch<N, T, MODE, TO, true, true>), grid, block, 0, s, bl);
  else hipLaunchKernelGGL((k_stencil_batch<N, T, MODE, TO, false, true>), grid, block, 0, s, bl);
  return hipGetLastError();
}

template <int N>
hipError_t launch_batch_order(int kind, bool gen, const BatchLaunch& bl, hipStream_t s) {
  switch (kind) {
    case K_F32_APPLY: return launch_batch_flavour<N, float, M_APPLY, float>(gen, bl, s);
    case K_F32_TRANSR: return launch_batch_flavour<N, float, M_TRANSR, float>(gen, bl, s);
    case K_F32_SUPD: return launch_batch_flavour<N, float, M_SUPD, float>(gen, bl, s);
    case K_F32_APPLY_EQ: return launch_batch_flavour<N, float, M_APPLY_EQ, float>(gen, bl, s);
    case K_F32_EQS: return launch_batch_flavour<N, float, M_EQS, float>(gen, bl, s);
    case K_F64_RESID32: return launch_batch_flavour<N, double, M_RESID, float>(gen, bl, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pn
