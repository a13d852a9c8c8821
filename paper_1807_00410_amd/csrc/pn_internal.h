// Internal declarations shared by the C-ABI translation units (not part of
// the public interface): the solver context and the host-side helpers that
// set up its padded geometry, pack vectors and dispatch the stencil kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "../../include/pn.h"
#include "../../include/pn_nn.h"
#include "pn_launch.h"
#include "pn_mg.h"

namespace pn {  // instantiated in pn_order_N.hip
extern template hipError_t launch_order<1>(int, bool, bool, const StencilArgs&, hipStream_t);
extern template hipError_t launch_order<2>(int, bool, bool, const StencilArgs&, hipStream_t);
extern template hipError_t launch_order<3>(int, bool, bool, const StencilArgs&, hipStream_t);
extern template hipError_t launch_order<4>(int, bool, bool, const StencilArgs&, hipStream_t);
extern template hipError_t launch_order<5>(int, bool, bool, const StencilArgs&, hipStream_t);
extern template hipError_t launch_order<6>(int, bool, bool, const StencilArgs&, hipStream_t);
extern template hipError_t launch_order<7>(int, bool, bool, const StencilArgs&, hipStream_t);
extern template hipError_t launch_lds_order<1>(int, bool, const StencilArgs&, hipStream_t);
extern template hipError_t launch_lds_order<2>(int, bool, const StencilArgs&, hipStream_t);
extern template hipError_t launch_lds_order<3>(int, bool, const StencilArgs&, hipStream_t);
extern template hipError_t launch_lds_order<4>(int, bool, const StencilArgs&, hipStream_t);
extern template hipError_t launch_lds_order<5>(int, bool, const StencilArgs&, hipStream_t);
extern template hipError_t launch_lds_order<6>(int, bool, const StencilArgs&, hipStream_t);
extern template hipError_t launch_lds_order<7>(int, bool, const StencilArgs&, hipStream_t);
extern template hipError_t lds_prepare<1>(size_t);
extern template hipError_t lds_prepare<2>(size_t);
extern template hipError_t lds_prepare<3>(size_t);
extern template hipError_t lds_prepare<4>(size_t);
extern template hipError_t lds_prepare<5>(size_t);
extern template hipError_t lds_prepare<6>(size_t);
extern template hipError_t lds_prepare<7>(size_t);
extern template hipError_t launch_batch_order<1>(int, bool, const BatchLaunch&, hipStream_t);
extern template hipError_t launch_batch_order<2>(int, bool, const BatchLaunch&, hipStream_t);
extern template hipError_t launch_batch_order<3>(int, bool, const BatchLaunch&, hipStream_t);
extern template hipError_t launch_batch_order<4>(int, bool, const BatchLaunch&, hipStream_t);
extern template hipError_t launch_batch_order<5>(int, bool, const BatchLaunch&, hipStream_t);
extern template hipError_t launch_batch_order<6>(int, bool, const BatchLaunch&, hipStream_t);
extern template hipError_t launch_batch_order<7>(int, bool, const BatchLaunch&, hipStream_t);
}  // namespace pn

using namespace pn;

struct pn_ctx {
  int order = 0, nc = 0;
  int nx = 0, ny = 0, nz = 0, bc = 0;
  int bcs[3] = {0, 0, 0};  // boundary type per axis (BC_VACUUM / BC_PERIODIC / BC_NEUMANN)
  bool zero_ext = false;   // some cell has zero extinction after the threshold (D_o singular)
  double h = 0.0;
  float g = 0.f, thr = 0.f;
  hipStream_t stream = nullptr;   // caller's stream
  hipStream_t sstream = nullptr;  // solve stream (graph capture needs a non-null stream)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  long n = 0;
  int off[kMaxCoeff] = {};
  int ext[kMaxCoeff][3] = {};
  int cls[kMaxCoeff][3] = {};
  float2* med = nullptr;    // padded cells (sigma_t thresholded, albedo)
  float2* med32 = nullptr;  // padded cells (sigma_a, sigma_s) FP32
  // padded lattice geometry (see StencilArgs)
  int PX = 0, PY = 0, plane = 0, CX = 0, cplane = 0;
  long long cs = 0, nv = 0;  // coefficient stride, padded vector length
  // FP32 Krylov workspace on the padded lattice (r ping-pong, s, p, q, d, rhs)
  float* r32[2] = {nullptr, nullptr};
  float *s32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr, *b32 = nullptr;
  double* x64 = nullptr;    // FP64 iterate (padded)
  uint16_t* m16 = nullptr;  // even-parity PCG preconditioner, bfloat16 (padded)
  // FP64 Krylov workspace, allocated on first use
  double* r64[2] = {nullptr, nullptr};
  double *s64 = nullptr, *p64 = nullptr, *q64 = nullptr, *d64 = nullptr;
  DevState* st = nullptr;
  DevState* st_host = nullptr;
  double* partials = nullptr;
  int* flag = nullptr;
  int* flag_host = nullptr;
  // launch geometry
  int Ex = 0, Ey = 0, Ez = 0;
  int zchunk = 0, nzc = 0, ncb = 0, nblocks = 0;
  int max_blocks = 0;
  // captured inner iterations
  hipGraphExec_t gexec32 = nullptr, gexec64 = nullptr;
  int giters32 = 0, giters64 = 0;
  // LDS-tiled FP32 stencil (vacuum boundary): tile shape and z chunking
  int lds_ok = 0;   // the tiled kernel fits this context
  int use_lds = 0;  // applies and the CG variant use it (opt-in, pn_set_tiles)
  int TX = 0, TY = 0, ntx = 0, nty = 0, lzchunk = 0, lnzc = 0, lnblocks = 0;
  size_t lds_bytes = 0, lds_max = 0;
  hipGraphExec_t gexec_schur = nullptr;  // captured even-parity PCG iterations
  int giters_schur = 0;
  EvenSlots even{};                   // even-band coefficient arrays of the padded vectors
  hipGraphExec_t gexec_cg = nullptr;  // captured CG-on-normal-equations iterations
  // multigrid preconditioner of the even-parity PCG (levels 1..mg_levels,
  // allocated on first use; geometry [0] = the class extents of the even slots)
  int mg_levels = 0;
  MgFine mg_fine{};
  MgGeom mg_geom[kMgMaxLevels] = {};
  MgTerms* mg_terms = nullptr;
  float4* mg_op[kMgMaxLevels] = {};
  float* mg_r[kMgMaxLevels] = {};
  float* mg_z[kMgMaxLevels] = {};
  float* mg_zt[kMgMaxLevels] = {};
  float* mg_idg[kMgMaxLevels] = {};  // 1 / diag per level (the same reciprocal every Jacobi step uses)
  double* mg_partials = nullptr;
  int mg_npart = 0;  // block partial pairs of <P^T r, V(P^T r)>
  int mg_tail_L0 = 0;  // first level of the one-launch tail of the V-cycle (0: none)
  MgTail* mg_tail = nullptr;
  int prec_ready = 0;  // bit 0: m16 formed, bit 1: the multigrid operators formed
  hipGraphExec_t gexec_mg = nullptr;
  int giters_mg = 0;
  int giters_cg = 0;
  int gcg_eq = 0;                     // gexec_cg holds the row-equilibrated form
  // learned initial guess / correction (pn_attach_net)
  pn_net* net = nullptr;
  uint16_t* net_x = nullptr;   // network input [cells8][32] bfloat16
  float* net_y = nullptr;      // network output [cells8][32]
  double* u64 = nullptr;       // network prediction on the padded lattice
  double* w64 = nullptr;       // A u
  unsigned* absmax = nullptr;  // max |source| (float bits)
  double* sq_part = nullptr;   // FP64 block partials (targets)
  DevState* st_net = nullptr;  // scalars of the learned step's line search (kept apart from st)
  std::string err;
};


#define PN_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) return fail(c, PN_ERR_HIP, std::string(#call) + ": " +  \
                                       hipGetErrorString(e_));                    \
  } while (0)

extern thread_local std::string g_setup_error;
pn_status fail(pn_ctx* c, pn_status s, const std::string& msg);
int grid_for(long n);
void set_geometry(pn_ctx* c, int zchunk);
StencilArgs base_args(const pn_ctx* c);
// Algorithmic bytes of the solve's kernels (vector elements read and written
// per unknown, the medium at 8 bytes per cell per stencil pass).
struct SolveBytes {
  double per_iter, per_start, per_resid;
};
inline SolveBytes solve_bytes(const pn_ctx* c, bool fp64, bool cg, bool eq) {
  const double n = (double)c->n, cells = (double)c->nx * c->ny * c->nz;
  SolveBytes b;
  if (fp64) {  // CGLS in FP64: A p (16), A^T r' with r' = r - alpha q (32), x/p update (40)
    b.per_iter = 88.0 * n + 16.0 * cells;
    b.per_start = 16.0 * n + 8.0 * cells + 32.0 * n;  // s = A^T r0, p = s, d = 0, x += d
  } else if (cg) {  // (W) A p (8), s -= alpha A^T q (12), x/p update (20)
    b.per_iter = 40.0 * n + 16.0 * cells;
    b.per_start = 8.0 * n + 8.0 * cells + 8.0 * n + 4.0 * n + 12.0 * n + (eq ? 8.0 * n + 8.0 * cells : 0.0);
  } else {  // CGLS: A p (8), r' = r - alpha q and A^T r' (16), x/p update (20)
    b.per_iter = 44.0 * n + 16.0 * cells;
    b.per_start = 8.0 * n + 8.0 * cells + 8.0 * n + 4.0 * n + 12.0 * n;
  }
  b.per_resid = 16.0 * n + 8.0 * cells;  // x FP64, Q, r
  return b;
}

// Even-parity PCG: per iteration the odd rows (read the even part of p,
// write the odd part), the even rows (read all of p, r and m in bfloat16,
// write r), x/p (x, p, r, m; write x, p); the medium per stencil pass.  With
// the multigrid preconditioner also: the restriction (read r), the level-1
// correction read by the x/p pass, and per coarse level the V-cycle's two
// passes (operator 16 B, r, z, z' per point) and the coarsest sweeps.
inline SolveBytes schur_bytes(const pn_ctx* c, bool mg = false) {
  double ne = 0.0;
  for (int j = 0; j < c->even.nk; ++j) {
    const int k = c->even.k[j];
    ne += (double)c->ext[k][0] * c->ext[k][1] * c->ext[k][2];
  }
  const double n = (double)c->n, no = n - ne, cells = (double)c->nx * c->ny * c->nz;
  SolveBytes b;
  b.per_iter = 4.0 * (ne + no) + (4.0 * n + 10.0 * ne) + 22.0 * ne + 16.0 * cells;
  if (mg && c->mg_levels > 0) {
    b.per_iter += 4.0 * ne + 4.0 * (double)c->mg_geom[1].off[c->mg_geom[1].nk];
    for (int L = 1; L <= c->mg_levels; ++L) {
      const double nl = (double)c->mg_geom[L].off[c->mg_geom[L].nk];
      b.per_iter += L < c->mg_levels ? nl * (16.0 + 4.0 + 4.0) + nl * (16.0 + 4.0 + 4.0 + 4.0) : nl * 24.0 * 16.0;
    }
  }
  b.per_start = 3.0 * n * 4.0 + 4.0 * ne * 4.0 + 16.0 * cells + (ne + n) * 4.0 + 12.0 * n;
  b.per_resid = 16.0 * n + 8.0 * cells;
  return b;
}

// Context with geometry and medium; the Krylov workspace only if `workspace`.
pn_status setup_ctx(int order, const pn_grid* grid, const pn_medium* med, void* stream, bool workspace,
                    pn_ctx** out);
// Mean milliseconds of one FP32 apply (register kernel, no reduction) for
// each zchunk candidate on padded vectors x -> y; sets the fastest and returns it.
int tune_zchunk(pn_ctx* c, const float* x, float* y, int iters, double* best_ms);
bool tune_lookup(const pn_ctx* c, int* zchunk, double* ms);
void tune_store(const pn_ctx* c, int zchunk, double ms);
void free_ctx(pn_ctx* c);
// The even-parity multigrid solve of the padded Q in c->b32 from the iterate
// in c->x64 (both set by the caller) on the context's solve stream (the
// batched solve's PN_VARIANT_SCHUR_MG path); o.variant must be SCHUR_MG.
pn_status solve_padded_mg(pn_ctx* c, double tol, const pn_solve_opts& o, pn_solve_info* info);
// True when the multigrid even-parity solve applies to the context.
bool mg_supported(const pn_ctx* c);
// Everything of the multigrid solve that allocates or captures (levels,
// coupling terms, the captured iteration graph for o.graph_iters), so that
// later solves of the context only launch work (needs the workspace).
pn_status prepare_mg_solve(pn_ctx* c, const pn_solve_opts& o);
// Points the FP32 scratch vectors (r0, r1, s, p, q, d) of a context created
// without workspace at caller-owned padded buffers v[0..5] and allocates the
// small owned parts (bfloat16 preconditioner, device scalars, partials) on
// first use; unborrow_workspace sets every borrowed pointer (and b32, x64)
// back to NULL.
pn_status borrow_workspace(pn_ctx* c, void* const* v);
void unborrow_workspace(pn_ctx* c);

inline PackArgs pack_args(const pn_ctx* c) {
  PackArgs p;
  std::memset(&p, 0, sizeof(p));
  p.nc = c->nc; p.PX = c->PX; p.PY = c->PY; p.plane = c->plane; p.cs = c->cs;
  for (int k = 0; k < c->nc; ++k) {
    p.off[k] = c->off[k];
    p.ex[k] = c->ext[k][0]; p.ey[k] = c->ext[k][1]; p.ez[k] = c->ext[k][2];
  }
  return p;
}


// DIR 0: padded <- packed; 1: packed <- padded; 2: packed += padded.
// launch_pack_args converts the coefficients of `pa` (a coefficient with
// ex = 0 is skipped).
template <typename TS, typename TD, int DIR>
inline hipError_t launch_pack_args(const pn_ctx* c, const PackArgs& pa, const TS* src, TD* dst, hipStream_t s) {
  long long maxsz = 0;
  for (int k = 0; k < c->nc; ++k) {
    long long sz = (long long)c->ext[k][0] * c->ext[k][1] * c->ext[k][2];
    if (sz > maxsz) maxsz = sz;
  }
  long long bx = (maxsz + kBlock - 1) / kBlock;
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL((k_pack<TS, TD, DIR>), dim3((unsigned)bx, c->nc), dim3(kBlock), 0, s, src, dst, pa);
  return hipGetLastError();
}
template <typename TS, typename TD, int DIR>
inline hipError_t launch_pack(const pn_ctx* c, const TS* src, TD* dst, hipStream_t s) {
  return launch_pack_args<TS, TD, DIR>(c, pack_args(c), src, dst, s);
}


// Dispatch on order (one translation unit per order) and boundary type; APPLY
// launches reduce ||y||^2 only when a.partials is set (the Krylov loop), the
// other modes always do.
template <typename T, int MODE, typename TO>
inline hipError_t launch_stencil(const pn_ctx* c, const StencilArgs& a, hipStream_t s) {
  const bool gen = c->bcs[0] != BC_VACUUM || c->bcs[1] != BC_VACUUM || c->bcs[2] != BC_VACUUM;
  const bool norm = !(MODE == M_APPLY && a.partials == nullptr);
  int kind;
  if constexpr (sizeof(T) == 4)
    kind = (MODE == M_APPLY) ? K_F32_APPLY
         : (MODE == M_SUPD) ? K_F32_SUPD
         : (MODE == M_APPLY_EQ) ? K_F32_APPLY_EQ
         : (MODE == M_EQS) ? K_F32_EQS
         : (MODE == M_ODD_W) ? K_F32_ODD_W
         : (MODE == M_EVEN_S) ? K_F32_EVEN_S
         : (MODE == M_EVEN_RHS) ? K_F32_EVEN_RHS
         : (MODE == M_ODD_BACK) ? K_F32_ODD_BACK
         : (MODE == M_EVEN_JAC) ? K_F32_EVEN_JAC
         : (MODE == M_EVEN_SR) ? K_F32_EVEN_SR : K_F32_TRANSR;
  else if constexpr (MODE == M_APPLY) kind = K_F64_APPLY;
  else if constexpr (MODE == M_TRANSR) kind = K_F64_TRANSR;
  else kind = (sizeof(TO) == 4) ? K_F64_RESID32 : K_F64_RESID64;
  switch (c->order) {
    case 1: return launch_order<1>(kind, gen, norm, a, s);
    case 2: return launch_order<2>(kind, gen, norm, a, s);
    case 3: return launch_order<3>(kind, gen, norm, a, s);
    case 4: return launch_order<4>(kind, gen, norm, a, s);
    case 5: return launch_order<5>(kind, gen, norm, a, s);
    case 6: return launch_order<6>(kind, gen, norm, a, s);
    case 7: return launch_order<7>(kind, gen, norm, a, s);
    default: return hipErrorInvalidValue;
  }
}

