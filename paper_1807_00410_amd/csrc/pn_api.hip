// C ABI of the staggered real P_N solver: context setup, matrix-free apply,
// FP64 residual and the mixed-precision CGLS solve (declarations and
// argument conventions in include/pn.h).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "../../include/pn.h"
#include "pn_kernels.h"

using namespace pn;

namespace {
thread_local std::string g_setup_error;
}

struct pn_ctx {
  int order = 0, nc = 0;
  int nx = 0, ny = 0, nz = 0, bc = 0;
  double h = 0.0;
  float g = 0.f, thr = 0.f;
  hipStream_t stream = nullptr;   // caller's stream
  hipStream_t sstream = nullptr;  // solve stream (graph capture needs a non-null stream)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  long n = 0;
  int off[kMaxCoeff] = {};
  int ext[kMaxCoeff][3] = {};
  int cls[kMaxCoeff][3] = {};
  float2* med = nullptr;
  // FP32 Krylov workspace (r ping-pong, s, p, q, d)
  float* r32[2] = {nullptr, nullptr};
  float *s32 = nullptr, *p32 = nullptr, *q32 = nullptr, *d32 = nullptr;
  // FP64 workspace, allocated on first use
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
  std::string err;
};

// ------------------------------------------------------------ utilities --
#define PN_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) return fail(c, PN_ERR_HIP, std::string(#call) + ": " +  \
                                       hipGetErrorString(e_));                    \
  } while (0)

static pn_status fail(pn_ctx* c, pn_status s, const std::string& msg) {
  if (c) c->err = msg; else g_setup_error = msg;
  return s;
}

static int grid_for(long n) {
  long b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

static void set_geometry(pn_ctx* c, int zchunk) {
  const int per = c->bc == PN_BC_PERIODIC;
  c->Ex = c->nx + (per ? 0 : 1);
  c->Ey = c->ny + (per ? 0 : 1);
  c->Ez = c->nz + (per ? 0 : 1);
  c->ncb = (c->Ex * c->Ey + kBlock - 1) / kBlock;
  if (zchunk <= 0) {
    // aim at ~2048 blocks (8 per CU), at least 4 planes per chunk
    int nzc = (2048 + c->ncb - 1) / c->ncb;
    zchunk = (c->Ez + nzc - 1) / nzc;
    if (zchunk < 4) zchunk = 4;
  }
  if (zchunk > c->Ez) zchunk = c->Ez;
  c->zchunk = zchunk;
  c->nzc = (c->Ez + zchunk - 1) / zchunk;
  c->nblocks = c->ncb * c->nzc;
}

static StencilArgs base_args(const pn_ctx* c) {
  StencilArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nx = c->nx; a.ny = c->ny; a.nz = c->nz;
  a.Ex = c->Ex; a.Ey = c->Ey; a.Ez = c->Ez;
  a.periodic = c->bc == PN_BC_PERIODIC;
  a.zchunk = c->zchunk; a.nzc = c->nzc; a.ncb = c->ncb; a.nblocks = c->nblocks;
  a.invh = 1.0 / c->h;
  a.tsign = 1.0;
  double gp = 1.0;
  for (int l = 0; l < 8; ++l) { a.omg[l] = 1.0 - gp; gp *= (double)c->g; }
  for (int k = 0; k < c->nc; ++k) a.off[k] = c->off[k];
  a.med = c->med;
  return a;
}

template <typename T, int MODE, typename TO>
static hipError_t launch_stencil(int order, const StencilArgs& a, hipStream_t s) {
  dim3 grid(a.nblocks), block(kBlock);
  switch (order) {
    case 1: hipLaunchKernelGGL((k_stencil<1, T, MODE, TO>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_stencil<2, T, MODE, TO>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_stencil<3, T, MODE, TO>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_stencil<4, T, MODE, TO>), grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_stencil<5, T, MODE, TO>), grid, block, 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_stencil<6, T, MODE, TO>), grid, block, 0, s, a); break;
    case 7: hipLaunchKernelGGL((k_stencil<7, T, MODE, TO>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static void free_all(pn_ctx* c) {
  if (!c) return;
  if (c->gexec32) hipGraphExecDestroy(c->gexec32);
  if (c->gexec64) hipGraphExecDestroy(c->gexec64);
  hipFree(c->med);
  for (int i = 0; i < 2; ++i) { hipFree(c->r32[i]); hipFree(c->r64[i]); }
  hipFree(c->s32); hipFree(c->p32); hipFree(c->q32); hipFree(c->d32);
  hipFree(c->s64); hipFree(c->p64); hipFree(c->q64); hipFree(c->d64);
  hipFree(c->st); hipFree(c->partials); hipFree(c->flag);
  if (c->st_host) hipHostFree(c->st_host);
  if (c->flag_host) hipHostFree(c->flag_host);
  if (c->ev_in) hipEventDestroy(c->ev_in);
  if (c->ev_out) hipEventDestroy(c->ev_out);
  if (c->sstream) hipStreamDestroy(c->sstream);
}

// ------------------------------------------------------------------ ABI --
extern "C" int pn_abi_version(void) { return PN_ABI_VERSION; }

extern "C" const char* pn_status_string(int s) {
  switch (s) {
    case PN_OK: return "ok";
    case PN_ERR_ARG: return "invalid argument";
    case PN_ERR_ALLOC: return "allocation failed";
    case PN_ERR_HIP: return "HIP runtime error";
    case PN_ERR_NONFINITE: return "non-finite input";
    case PN_ERR_NOT_CONVERGED: return "not converged";
    case PN_ERR_BREAKDOWN: return "Krylov breakdown";
    default: return "unknown status";
  }
}

extern "C" void pn_default_opts(pn_solve_opts* o) {
  if (!o) return;
  o->precision = PN_FP32_IR;
  o->max_iter = 200000;
  o->max_refine = 40;
  o->inner_tol = 1e-3;
  o->use_guess = 0;
  o->graph_iters = 32;
}

extern "C" const char* pn_last_error(const pn_ctx* c) {
  return c ? c->err.c_str() : g_setup_error.c_str();
}

extern "C" pn_status pn_setup(int order, const pn_grid* grid, const pn_medium* med, void* stream,
                              pn_ctx** out) {
  pn_ctx* c = nullptr;
  if (!out) return fail(nullptr, PN_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (order < 1 || order > PN_MAX_ORDER) return fail(nullptr, PN_ERR_ARG, "order must be in 1..7");
  if (!grid || !med) return fail(nullptr, PN_ERR_ARG, "grid or medium is NULL");
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return fail(nullptr, PN_ERR_ARG, "grid dimensions must be >= 1");
  if (grid->bc != PN_BC_VACUUM && grid->bc != PN_BC_PERIODIC) return fail(nullptr, PN_ERR_ARG, "unknown boundary type");
  if (!med->sigma_t || !med->albedo) return fail(nullptr, PN_ERR_ARG, "medium arrays are NULL");
  if (!(med->g > -1.f && med->g < 1.f)) return fail(nullptr, PN_ERR_ARG, "g must be in (-1, 1)");
  if (!(med->sigma_t_min >= 0.f) || !std::isfinite(med->sigma_t_min)) return fail(nullptr, PN_ERR_ARG, "sigma_t_min must be finite and >= 0");
  const long cells = (long)grid->nx * grid->ny * grid->nz;
  if (cells > (1L << 30)) return fail(nullptr, PN_ERR_ARG, "grid too large");

  c = new pn_ctx();
  c->order = order;
  c->nc = (order + 1) * (order + 1);
  c->nx = grid->nx; c->ny = grid->ny; c->nz = grid->nz; c->bc = grid->bc;
  c->h = grid->h > 0.0 ? grid->h : 1.0 / grid->nx;
  c->g = med->g;
  c->thr = med->sigma_t_min;
  c->stream = (hipStream_t)stream;
  long n = 0;
  const int per = c->bc == PN_BC_PERIODIC;
  for (int k = 0; k < c->nc; ++k) {
    int p[3];
    int l = 0;
    while ((l + 1) * (l + 1) <= k) ++l;
    const int m = k - l * l - l, am = m < 0 ? -m : m;
    p[0] = m >= 0 ? (m & 1) : ((am + 1) & 1);
    p[1] = m < 0 ? 1 : 0;
    p[2] = (l + am) & 1;
    const int dims[3] = {c->nx, c->ny, c->nz};
    long sz = 1;
    for (int d = 0; d < 3; ++d) {
      c->cls[k][d] = p[d];
      c->ext[k][d] = dims[d] + (per ? 0 : p[d]);
      sz *= c->ext[k][d];
    }
    c->off[k] = (int)n;
    n += sz;
    if (n >= (1L << 31) - 1) { delete c; return fail(nullptr, PN_ERR_ARG, "too many unknowns (>= 2^31)"); }
  }
  c->n = n;
  set_geometry(c, 0);
  c->max_blocks = 1 << 16;
  if (c->nblocks > c->max_blocks) { delete c; return fail(nullptr, PN_ERR_ARG, "grid too large in x*y"); }

  auto bail = [&](pn_status s, const std::string& m) {
    free_all(c);
    delete c;
    return fail(nullptr, s, m);
  };
#define SETUP_HIP(call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) return bail(e_ == hipErrorOutOfMemory ? PN_ERR_ALLOC : PN_ERR_HIP, \
                                      std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

  SETUP_HIP(hipStreamCreateWithFlags(&c->sstream, hipStreamNonBlocking));
  SETUP_HIP(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
  SETUP_HIP(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
  SETUP_HIP(hipMalloc(&c->med, sizeof(float2) * cells));
  for (int i = 0; i < 2; ++i) SETUP_HIP(hipMalloc(&c->r32[i], sizeof(float) * n));
  SETUP_HIP(hipMalloc(&c->s32, sizeof(float) * n));
  SETUP_HIP(hipMalloc(&c->p32, sizeof(float) * n));
  SETUP_HIP(hipMalloc(&c->q32, sizeof(float) * n));
  SETUP_HIP(hipMalloc(&c->d32, sizeof(float) * n));
  SETUP_HIP(hipMalloc(&c->st, sizeof(DevState)));
  SETUP_HIP(hipHostMalloc(&c->st_host, sizeof(DevState), hipHostMallocDefault));
  SETUP_HIP(hipMalloc(&c->partials, sizeof(double) * 2 * c->max_blocks));
  SETUP_HIP(hipMalloc(&c->flag, sizeof(int)));
  SETUP_HIP(hipHostMalloc(&c->flag_host, sizeof(int), hipHostMallocDefault));

  SETUP_HIP(hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
  hipLaunchKernelGGL(k_medium_prep, dim3(grid_for(cells)), dim3(kBlock), 0, c->stream, med->sigma_t,
                     med->albedo, c->thr, c->med, cells, c->flag);
  SETUP_HIP(hipGetLastError());
  SETUP_HIP(hipMemcpyAsync(c->flag_host, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  SETUP_HIP(hipStreamSynchronize(c->stream));
  if (*c->flag_host) return bail(PN_ERR_NONFINITE, "medium contains NaN or Inf");
#undef SETUP_HIP
  *out = c;
  return PN_OK;
}

extern "C" pn_status pn_set_zchunk(pn_ctx* c, int zchunk) {
  if (!c) return PN_ERR_ARG;
  if (zchunk < 0) return fail(c, PN_ERR_ARG, "zchunk must be >= 0");
  set_geometry(c, zchunk);
  if (c->nblocks > c->max_blocks) { set_geometry(c, 0); return fail(c, PN_ERR_ARG, "too many blocks"); }
  if (c->gexec32) { hipGraphExecDestroy(c->gexec32); c->gexec32 = nullptr; c->giters32 = 0; }
  if (c->gexec64) { hipGraphExecDestroy(c->gexec64); c->gexec64 = nullptr; c->giters64 = 0; }
  return PN_OK;
}

extern "C" int pn_get_zchunk(const pn_ctx* c) { return c ? c->zchunk : -1; }

extern "C" pn_status pn_layout_query(const pn_ctx* c, pn_layout* L) {
  if (!c || !L) return PN_ERR_ARG;
  std::memset(L, 0, sizeof(*L));
  L->order = c->order; L->ncoeff = c->nc;
  L->nx = c->nx; L->ny = c->ny; L->nz = c->nz; L->bc = c->bc;
  L->n_unknowns = c->n;
  for (int k = 0; k < c->nc; ++k) {
    for (int d = 0; d < 3; ++d) { L->cls[k][d] = c->cls[k][d]; L->ext[k][d] = c->ext[k][d]; }
    L->offset[k] = c->off[k];
  }
  L->offset[c->nc] = c->n;
  return PN_OK;
}

extern "C" pn_status pn_apply(pn_ctx* c, const float* x, float* y, int transpose) {
  if (!c) return PN_ERR_ARG;
  if (!x || !y) return fail(c, PN_ERR_ARG, "x or y is NULL");
  if ((const void*)x == (const void*)y) return fail(c, PN_ERR_ARG, "x and y must not alias");
  StencilArgs a = base_args(c);
  a.tsign = transpose ? -1.0 : 1.0;
  a.x = x; a.y = y;
  PN_HIP((launch_stencil<float, M_APPLY, float>(c->order, a, c->stream)));
  return PN_OK;
}

extern "C" pn_status pn_apply64(pn_ctx* c, const double* x, double* y, int transpose) {
  if (!c) return PN_ERR_ARG;
  if (!x || !y) return fail(c, PN_ERR_ARG, "x or y is NULL");
  if ((const void*)x == (const void*)y) return fail(c, PN_ERR_ARG, "x and y must not alias");
  StencilArgs a = base_args(c);
  a.tsign = transpose ? -1.0 : 1.0;
  a.x = x; a.y = y;
  PN_HIP((launch_stencil<double, M_APPLY, double>(c->order, a, c->stream)));
  return PN_OK;
}

static pn_status ensure64(pn_ctx* c) {
  if (c->s64) return PN_OK;
  const size_t b = sizeof(double) * c->n;
  for (int i = 0; i < 2; ++i) PN_HIP(hipMalloc(&c->r64[i], b));
  PN_HIP(hipMalloc(&c->s64, b));
  PN_HIP(hipMalloc(&c->p64, b));
  PN_HIP(hipMalloc(&c->q64, b));
  PN_HIP(hipMalloc(&c->d64, b));
  return PN_OK;
}

// r = Q - A x in FP64 arithmetic; r stored as TO; partials -> st->rtrue2, st->bb2.
template <typename TO>
static pn_status residual(pn_ctx* c, const float* rhs, const double* x, TO* r, hipStream_t s) {
  StencilArgs a = base_args(c);
  a.x = x; a.x2 = rhs; a.y = r;
  a.partials = c->partials;
  PN_HIP((launch_stencil<double, M_RESID, TO>(c->order, a, s)));
  hipLaunchKernelGGL(k_fin_resid, dim3(1), dim3(kBlock), 0, s, c->st, c->partials, c->nblocks);
  PN_HIP(hipGetLastError());
  return PN_OK;
}

extern "C" pn_status pn_residual64(pn_ctx* c, const float* rhs, const double* x, double* r, double* rel) {
  if (!c) return PN_ERR_ARG;
  if (!rhs || !x) return fail(c, PN_ERR_ARG, "rhs or x is NULL");
  pn_status s = PN_OK;
  if (!r) {
    s = ensure64(c);
    if (s != PN_OK) return s;
    r = c->r64[0];
  }
  s = residual<double>(c, rhs, x, r, c->stream);
  if (s != PN_OK) return s;
  PN_HIP(hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
  PN_HIP(hipStreamSynchronize(c->stream));
  if (rel) *rel = c->st_host->bb2 > 0.0 ? std::sqrt(c->st_host->rtrue2 / c->st_host->bb2) : 0.0;
  return PN_OK;
}

// One CGLS iteration on vectors of type T (r ping-pong rin -> rout).
template <typename T>
static hipError_t enqueue_iteration(pn_ctx* c, T* d, T* p, T* q, T* s, const T* rin, T* rout, hipStream_t st) {
  StencilArgs a = base_args(c);
  a.st = c->st;
  a.partials = c->partials;
  a.x = p; a.y = q; a.tsign = 1.0;
  hipError_t e = launch_stencil<T, M_APPLY, T>(c->order, a, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(kBlock), 0, st, c->st, c->partials, c->nblocks);
  a.x = rin; a.x2 = q; a.y = s; a.y2 = rout; a.tsign = -1.0;
  e = launch_stencil<T, M_TRANSR, T>(c->order, a, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fin_beta, dim3(1), dim3(kBlock), 0, st, c->st, c->partials, c->nblocks);
  hipLaunchKernelGGL((k_update_xp<T>), dim3(grid_for(c->n / (sizeof(T) == 4 ? 4 : 1) + 1)), dim3(kBlock), 0, st,
                     d, p, (const T*)s, c->n, (const DevState*)c->st);
  return hipGetLastError();
}

template <typename T>
static pn_status build_graph(pn_ctx* c, int iters, T* d, T* p, T* q, T* s, T* r0, T* r1,
                             hipGraphExec_t* exec) {
  hipGraph_t g = nullptr;
  PN_HIP(hipStreamBeginCapture(c->sstream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int i = 0; i < iters && e == hipSuccess; ++i)
    e = (i & 1) ? enqueue_iteration<T>(c, d, p, q, s, r1, r0, c->sstream)
                : enqueue_iteration<T>(c, d, p, q, s, r0, r1, c->sstream);
  hipError_t e2 = hipStreamEndCapture(c->sstream, &g);
  if (e != hipSuccess) { if (g) hipGraphDestroy(g); return fail(c, PN_ERR_HIP, std::string("capture: ") + hipGetErrorString(e)); }
  if (e2 != hipSuccess) return fail(c, PN_ERR_HIP, std::string("end capture: ") + hipGetErrorString(e2));
  hipError_t e3 = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e3 != hipSuccess) return fail(c, PN_ERR_HIP, std::string("instantiate: ") + hipGetErrorString(e3));
  return PN_OK;
}

template <typename T>
static pn_status solve_impl(pn_ctx* c, const float* rhs, double* x, double tol, const pn_solve_opts& o,
                            pn_solve_info* info) {
  T *r0, *r1, *s, *p, *q, *d;
  hipGraphExec_t* gexec;
  int* giters;
  if constexpr (sizeof(T) == 4) {
    r0 = c->r32[0]; r1 = c->r32[1]; s = c->s32; p = c->p32; q = c->q32; d = c->d32;
    gexec = &c->gexec32; giters = &c->giters32;
  } else {
    pn_status e = ensure64(c);
    if (e != PN_OK) return e;
    r0 = c->r64[0]; r1 = c->r64[1]; s = c->s64; p = c->p64; q = c->q64; d = c->d64;
    gexec = &c->gexec64; giters = &c->giters64;
  }
  int gi = o.graph_iters < 2 ? 2 : (o.graph_iters + 1) & ~1;  // even: r ends in r0
  if (*gexec == nullptr || *giters != gi) {
    if (*gexec) { hipGraphExecDestroy(*gexec); *gexec = nullptr; }
    pn_status e = build_graph<T>(c, gi, d, p, q, s, r0, r1, gexec);
    if (e != PN_OK) return e;
    *giters = gi;
  }
  hipStream_t ss = c->sstream;
  DevState init;
  std::memset(&init, 0, sizeof(init));
  init.max_iters = o.max_iter;
  PN_HIP(hipMemcpyAsync(c->st, &init, sizeof(DevState), hipMemcpyHostToDevice, ss));
  PN_HIP(hipStreamSynchronize(ss));
  if (!o.use_guess) {
    hipLaunchKernelGGL((k_fill<double>), dim3(grid_for(c->n)), dim3(kBlock), 0, ss, x, c->n, 0.0);
    PN_HIP(hipGetLastError());
  }
  pn_status result = PN_ERR_NOT_CONVERGED;
  int outer = 0;
  double rel = 0.0, bnorm = 0.0;
  if (info) info->nhistory = 0;
  for (;;) {
    pn_status e = residual<T>(c, rhs, x, r0, ss);
    if (e != PN_OK) return e;
    PN_HIP(hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, ss));
    PN_HIP(hipStreamSynchronize(ss));
    const DevState h = *c->st_host;
    ++outer;
    bnorm = std::sqrt(h.bb2);
    if (h.bb2 == 0.0) {  // Q = 0: the solution is 0
      hipLaunchKernelGGL((k_fill<double>), dim3(grid_for(c->n)), dim3(kBlock), 0, ss, x, c->n, 0.0);
      PN_HIP(hipGetLastError());
      rel = 0.0;
      result = PN_OK;
      break;
    }
    rel = std::sqrt(h.rtrue2 / h.bb2);
    if (info && info->nhistory < PN_MAX_HISTORY) info->history[info->nhistory++] = rel;
    if (!std::isfinite(rel)) { result = PN_ERR_NONFINITE; break; }
    if (rel <= tol) { result = PN_OK; break; }
    if (outer > o.max_refine || h.iters >= o.max_iter) { result = PN_ERR_NOT_CONVERGED; break; }
    if (h.breakdown) { result = PN_ERR_BREAKDOWN; break; }
    // inner solve  A d = r0  from d = 0
    double itol = o.inner_tol;
    if constexpr (sizeof(T) == 8) itol = 0.5 * tol / rel;  // FP64: go all the way
    if (itol >= 1.0) itol = 0.5;
    hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(c->n)), dim3(kBlock), 0, ss, d, c->n, T(0));
    StencilArgs a = base_args(c);
    a.x = r0; a.y = s; a.y2 = p; a.tsign = -1.0; a.partials = c->partials;
    PN_HIP((launch_stencil<T, M_APPLY, T>(c->order, a, ss)));
    hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(kBlock), 0, ss, c->st, c->partials, c->nblocks, itol * itol);
    PN_HIP(hipGetLastError());
    for (;;) {
      PN_HIP(hipGraphLaunch(*gexec, ss));
      PN_HIP(hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, ss));
      PN_HIP(hipStreamSynchronize(ss));
      if (c->st_host->done || c->st_host->stop) break;
    }
    // the last graph may have stopped with stop set but done unset: x update already applied
    hipLaunchKernelGGL((k_add_to64<T>), dim3(grid_for(c->n)), dim3(kBlock), 0, ss, x, (const T*)d, c->n);
    PN_HIP(hipGetLastError());
  }
  if (info) {
    info->status = result;
    info->outer_iters = outer;
    info->inner_iters = c->st_host->iters;
    info->rel_residual = rel;
    info->bnorm = bnorm;
  }
  return result;
}

extern "C" pn_status pn_solve(pn_ctx* c, const float* rhs, double* x, double tol, const pn_solve_opts* opts,
                              pn_solve_info* info) {
  if (!c) return PN_ERR_ARG;
  if (!rhs || !x) return fail(c, PN_ERR_ARG, "rhs or x is NULL");
  if (!(tol > 0.0)) return fail(c, PN_ERR_ARG, "tol must be > 0");
  pn_solve_opts o;
  pn_default_opts(&o);
  if (opts) o = *opts;
  if (o.max_iter < 1 || o.max_refine < 0 || !(o.inner_tol > 0.0 && o.inner_tol < 1.0))
    return fail(c, PN_ERR_ARG, "invalid solve options");
  if (o.precision != PN_FP32_IR && o.precision != PN_FP64) return fail(c, PN_ERR_ARG, "unknown precision");
  if (info) std::memset(info, 0, sizeof(*info));
  const auto t0 = std::chrono::steady_clock::now();
  // order the solve after the caller's pending work
  PN_HIP(hipEventRecord(c->ev_in, c->stream));
  PN_HIP(hipStreamWaitEvent(c->sstream, c->ev_in, 0));
  // non-finite right-hand side
  PN_HIP(hipMemsetAsync(c->flag, 0, sizeof(int), c->sstream));
  hipLaunchKernelGGL(k_check_finite, dim3(grid_for(c->n)), dim3(kBlock), 0, c->sstream, rhs, c->n, c->flag);
  PN_HIP(hipGetLastError());
  PN_HIP(hipMemcpyAsync(c->flag_host, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->sstream));
  PN_HIP(hipStreamSynchronize(c->sstream));
  if (*c->flag_host) return fail(c, PN_ERR_NONFINITE, "right-hand side contains NaN or Inf");
  pn_status s = (o.precision == PN_FP64) ? solve_impl<double>(c, rhs, x, tol, o, info)
                                          : solve_impl<float>(c, rhs, x, tol, o, info);
  PN_HIP(hipEventRecord(c->ev_out, c->sstream));
  PN_HIP(hipStreamWaitEvent(c->stream, c->ev_out, 0));
  PN_HIP(hipStreamSynchronize(c->sstream));
  if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (s == PN_ERR_NOT_CONVERGED) fail(c, s, "tolerance not reached within max_iter / max_refine");
  if (s == PN_ERR_BREAKDOWN) fail(c, s, "CGLS breakdown");
  if (s == PN_ERR_NONFINITE) fail(c, s, "non-finite residual");
  return s;
}

extern "C" void pn_destroy(pn_ctx* c) {
  if (!c) return;
  if (c->sstream) hipStreamSynchronize(c->sstream);
  if (c->stream) hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
}

// Coupling table of the compiled operator (for host-side checks):
// fills up to `cap` entries (k, d, k', value) and returns the total count.
template <int N>
static int copy_table(int* k, int* d, int* kp, double* v, int cap) {
  using TB = Table<N>;
  for (int i = 0; i < TB::NCPL && i < cap; ++i) {
    k[i] = TB::cpl.v[i].k; d[i] = TB::cpl.v[i].d; kp[i] = TB::cpl.v[i].kp; v[i] = TB::cpl.v[i].c;
  }
  return TB::NCPL;
}

extern "C" int pn_coupling_table(int order, int* k, int* d, int* kp, double* v, int cap) {
  if (!k || !d || !kp || !v || cap < 0) return -1;
  switch (order) {
    case 1: return copy_table<1>(k, d, kp, v, cap);
    case 2: return copy_table<2>(k, d, kp, v, cap);
    case 3: return copy_table<3>(k, d, kp, v, cap);
    case 4: return copy_table<4>(k, d, kp, v, cap);
    case 5: return copy_table<5>(k, d, kp, v, cap);
    case 6: return copy_table<6>(k, d, kp, v, cap);
    case 7: return copy_table<7>(k, d, kp, v, cap);
    default: return -1;
  }
}
