// C ABI of the staggered real P_N solver: context setup, matrix-free apply,
// FP64 residual and the mixed-precision CGLS solve (declarations and
// argument conventions in include/pn.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pn.h"
#include "pn_internal.h"
#include "pn_render.h"
#include "pn_mg_kernels.h"
#include "pn_learned.h"


using namespace pn;

thread_local std::string g_setup_error;


static constexpr size_t kLdsMax = 160 * 1024;

// Tile geometry of the LDS kernel; returns false if the shape is not usable.
static bool set_tiles(pn_ctx* c, int TX, int TY, int zchunk) {
  if (c->bcs[0] != BC_VACUUM || c->bcs[1] != BC_VACUUM || c->bcs[2] != BC_VACUUM || TX < 1 || TY < 1) return false;
  const int threads = ((TX * TY + 63) / 64) * 64;
  if (threads > kBlock || 2 * (TX + 2) + 2 * TY > threads) return false;
  const size_t bytes = sizeof(float) * (size_t)c->nc * (TX + 2) * (TY + 2);
  if (bytes > c->lds_max) return false;
  const int ntx = (c->Ex + TX - 1) / TX, nty = (c->Ey + TY - 1) / TY;
  if (zchunk <= 0) {  // about 8 blocks per CU, at least 4 planes per chunk
    const int nzc = (2048 + ntx * nty - 1) / (ntx * nty);
    zchunk = (c->Ez + nzc - 1) / nzc;
    if (zchunk < 4) zchunk = 4;
  }
  if (zchunk > c->Ez) zchunk = c->Ez;
  const int lnzc = (c->Ez + zchunk - 1) / zchunk;
  if ((long long)ntx * nty * lnzc > c->max_blocks) return false;
  c->TX = TX; c->TY = TY; c->ntx = ntx; c->nty = nty;
  c->lzchunk = zchunk; c->lnzc = lnzc; c->lnblocks = ntx * nty * lnzc;
  c->lds_bytes = bytes;
  return true;
}

// Default tile: least lanes per lattice column (idle lanes and halo reloads
// weighted), rows of at least 32 columns for coalescing, and preferring shapes
// whose LDS lets two blocks share a CU.
static void choose_tiles(pn_ctx* c) {
  double best = 1e30;
  int bx = 0, by = 0;
  const int txmin = c->Ex < 32 ? c->Ex : 32;
  for (int TX = txmin; TX <= (c->Ex < kBlock ? c->Ex : kBlock); ++TX)
    for (int TY = 1; TX * TY <= kBlock; ++TY) {
      const int threads = ((TX * TY + 63) / 64) * 64;
      if (2 * (TX + 2) + 2 * TY > threads) continue;
      const size_t bytes = sizeof(float) * (size_t)c->nc * (TX + 2) * (TY + 2);
      if (bytes > c->lds_max) continue;
      const double lanes = (double)((c->Ex + TX - 1) / TX) * ((c->Ey + TY - 1) / TY) * threads;
      const double waste = lanes / ((double)c->Ex * c->Ey);
      const double halo = (double)((TX + 2) * (TY + 2) - TX * TY) / (TX * TY);
      const double cost = waste * (1.0 + 0.25 * halo) * (2 * bytes <= kLdsMax ? 1.0 : 1.15);
      if (cost < best) { best = cost; bx = TX; by = TY; }
    }
  c->lds_ok = (bx > 0) && set_tiles(c, bx, by, 0);
}


// LDS-tiled FP32 apply: mode M_APPLY (norm optional) or M_SUPD.
static hipError_t launch_lds(const pn_ctx* c, int mode, bool norm, StencilArgs a, hipStream_t s) {
  a.TX = c->TX; a.TY = c->TY; a.ntx = c->ntx; a.nty = c->nty;
  a.zchunk = c->lzchunk; a.nzc = c->lnzc; a.nblocks = c->lnblocks;
  switch (c->order) {
    case 1: return launch_lds_order<1>(mode, norm, a, s);
    case 2: return launch_lds_order<2>(mode, norm, a, s);
    case 3: return launch_lds_order<3>(mode, norm, a, s);
    case 4: return launch_lds_order<4>(mode, norm, a, s);
    case 5: return launch_lds_order<5>(mode, norm, a, s);
    case 6: return launch_lds_order<6>(mode, norm, a, s);
    case 7: return launch_lds_order<7>(mode, norm, a, s);
    default: return hipErrorInvalidValue;
  }
}

static hipError_t lds_prepare_order(int order, size_t bytes) {
  switch (order) {
    case 1: return lds_prepare<1>(bytes);
    case 2: return lds_prepare<2>(bytes);
    case 3: return lds_prepare<3>(bytes);
    case 4: return lds_prepare<4>(bytes);
    case 5: return lds_prepare<5>(bytes);
    case 6: return lds_prepare<6>(bytes);
    case 7: return lds_prepare<7>(bytes);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------ utilities --

pn_status fail(pn_ctx* c, pn_status s, const std::string& msg) {
  if (c) c->err = msg; else g_setup_error = msg;
  return s;
}

// One thread per element of a streaming update (no grid-stride cap: ~4%
// faster on the 81M-element x/p update than 8192 blocks striding).
static int stream_grid(long n) {
  long b = (n + kBlock - 1) / kBlock;
  return (int)(b < 1 ? 1 : b);
}

int grid_for(long n) {
  long b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

void set_geometry(pn_ctx* c, int zchunk) {
  c->Ex = c->nx + (c->bcs[0] == BC_PERIODIC ? 0 : 1);
  c->Ey = c->ny + (c->bcs[1] == BC_PERIODIC ? 0 : 1);
  c->Ez = c->nz + (c->bcs[2] == BC_PERIODIC ? 0 : 1);
  c->PX = c->Ex + 2;
  c->PY = c->Ey + 2;
  c->plane = c->PX * c->PY;
  c->CX = c->nx + 2;
  c->cplane = c->CX * (c->ny + 2);
  c->cs = (((long long)c->plane * (c->Ez + 2)) + 63) / 64 * 64;
  c->nv = c->cs * c->nc;
  c->even.cs = c->cs;
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

StencilArgs base_args(const pn_ctx* c) {
  StencilArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nx = c->nx; a.ny = c->ny; a.nz = c->nz;
  a.Ex = c->Ex; a.Ey = c->Ey; a.Ez = c->Ez;
  a.PX = c->PX; a.PY = c->PY; a.plane = c->plane;
  a.CX = c->CX; a.cplane = c->cplane;
  a.cs = c->cs;
  a.zchunk = c->zchunk; a.nzc = c->nzc; a.ncb = c->ncb; a.nblocks = c->nblocks;
  a.bcx = c->bcs[0]; a.bcy = c->bcs[1]; a.bcz = c->bcs[2];
  a.invh = 1.0 / c->h;
  a.tsign = 1.0;
  double gp = 1.0;
  for (int l = 0; l < 8; ++l) { a.omg[l] = 1.0 - gp; gp *= (double)c->g; }
  a.med = c->med;
  a.med32 = c->med32;
  return a;
}




static void free_all(pn_ctx* c) {
  if (!c) return;
  if (c->gexec32) hipGraphExecDestroy(c->gexec32);
  if (c->gexec64) hipGraphExecDestroy(c->gexec64);
  if (c->gexec_cg) hipGraphExecDestroy(c->gexec_cg);
  if (c->gexec_schur) hipGraphExecDestroy(c->gexec_schur);
  if (c->gexec_mg) hipGraphExecDestroy(c->gexec_mg);
  hipFree(c->mg_terms);
  hipFree(c->mg_partials);
  hipFree(c->mg_tail);
  for (int L = 0; L < kMgMaxLevels; ++L) {
    hipFree(c->mg_op[L]); hipFree(c->mg_r[L]); hipFree(c->mg_z[L]); hipFree(c->mg_zt[L]); hipFree(c->mg_idg[L]);
  }
  hipFree(c->med); hipFree(c->med32);
  for (int i = 0; i < 2; ++i) { hipFree(c->r32[i]); hipFree(c->r64[i]); }
  hipFree(c->m16);
  hipFree(c->s32); hipFree(c->p32); hipFree(c->q32); hipFree(c->d32); hipFree(c->b32); hipFree(c->x64);
  hipFree(c->s64); hipFree(c->p64); hipFree(c->q64); hipFree(c->d64);
  hipFree(c->st); hipFree(c->partials); hipFree(c->flag);
  hipFree(c->net_x); hipFree(c->net_y); hipFree(c->u64); hipFree(c->w64); hipFree(c->absmax); hipFree(c->sq_part);
  hipFree(c->st_net);
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
  o->inner_tol = 1e-2;
  o->use_guess = 0;
  o->graph_iters = 8;  // measured: 8 per graph is 0.8% (P5 128^3) to 5% (batched workload) faster than 32
  o->variant = PN_VARIANT_AUTO;
  o->learned = PN_LEARNED_OFF;
}

extern "C" const char* pn_last_error(const pn_ctx* c) {
  return c ? c->err.c_str() : g_setup_error.c_str();
}

// ------------------------------------------------------------- autotuner --
// Launch tuning of the register-window stencil: the number of z planes a
// block marches (zchunk) trades launch width against the re-read of the
// window planes at chunk borders.  Candidates are timed on the device and the
// fastest is kept in a process-wide cache keyed by (order, grid, boundary),
// which contexts consult at setup and which can be saved to / loaded from a
// text file.
namespace {
struct TuneKey {
  int order, nx, ny, nz, bc;
  bool operator<(const TuneKey& o) const {
    return std::tie(order, nx, ny, nz, bc) < std::tie(o.order, o.nx, o.ny, o.nz, o.bc);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, double>> g_tune;
// boundary part of the key: bc_x + 3 bc_y + 9 bc_z (0: vacuum everywhere)
TuneKey key_of(const pn_ctx* c) {
  return TuneKey{c->order, c->nx, c->ny, c->nz, c->bcs[0] + 3 * c->bcs[1] + 9 * c->bcs[2]};
}
}  // namespace

bool tune_lookup(const pn_ctx* c, int* zchunk, double* ms) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(key_of(c));
  if (it == g_tune.end()) return false;
  if (zchunk) *zchunk = it->second.first;
  if (ms) *ms = it->second.second;
  return true;
}

void tune_store(const pn_ctx* c, int zchunk, double ms) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key_of(c)] = {zchunk, ms};
}

int tune_zchunk(pn_ctx* c, const float* x, float* y, int iters, double* best_ms) {
  static const int cand[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 24, 32};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int best = c->zchunk;
  double bms = -1.0;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return -1;
  }
  bool ok = true;
  for (int z : cand) {
    if (z > c->Ez && z != cand[0]) break;
    set_geometry(c, z);
    if (c->nblocks > c->max_blocks) continue;
    StencilArgs a = base_args(c);
    a.x = x; a.y = y;
    ok = ok && launch_stencil<float, M_APPLY, float>(c, a, c->stream) == hipSuccess;  // warm-up
    ok = ok && hipEventRecord(e0, c->stream) == hipSuccess;
    for (int i = 0; i < iters && ok; ++i) ok = launch_stencil<float, M_APPLY, float>(c, a, c->stream) == hipSuccess;
    ok = ok && hipEventRecord(e1, c->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.f;
    ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    if (!ok) break;
    const double per = (double)ms / iters;
    if (bms < 0.0 || per < bms) { bms = per; best = c->zchunk; }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  set_geometry(c, best);
  if (!ok) return -1;
  if (best_ms) *best_ms = bms;
  return best;
}

extern "C" pn_status pn_autotune(pn_ctx* c, int iters, int* zchunk, double* ms) {
  if (!c) return PN_ERR_ARG;
  if (iters < 1) return fail(c, PN_ERR_ARG, "iters must be >= 1");
  if (!c->p32) return fail(c, PN_ERR_ARG, "context has no workspace");
  double bms = 0.0;
  const int z = tune_zchunk(c, c->p32, c->q32, iters, &bms);
  if (z < 0) return fail(c, PN_ERR_HIP, "autotune: a timing launch failed");
  tune_store(c, z, bms);
  if (c->gexec32) { hipGraphExecDestroy(c->gexec32); c->gexec32 = nullptr; c->giters32 = 0; }
  if (c->gexec64) { hipGraphExecDestroy(c->gexec64); c->gexec64 = nullptr; c->giters64 = 0; }
  if (c->gexec_cg) { hipGraphExecDestroy(c->gexec_cg); c->gexec_cg = nullptr; c->giters_cg = 0; }
  if (c->gexec_schur) { hipGraphExecDestroy(c->gexec_schur); c->gexec_schur = nullptr; c->giters_schur = 0; }
  if (c->gexec_mg) { hipGraphExecDestroy(c->gexec_mg); c->gexec_mg = nullptr; c->giters_mg = 0; }
  if (zchunk) *zchunk = z;
  if (ms) *ms = bms;
  return PN_OK;
}

extern "C" int pn_tune_cache_size(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return (int)g_tune.size();
}

extern "C" void pn_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

extern "C" pn_status pn_tune_cache_save(const char* path) {
  if (!path) return PN_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return PN_ERR_ARG;
  std::fprintf(f, "# pn stencil tune cache: order nx ny nz bc zchunk ms\n");
  for (const auto& kv : g_tune)
    std::fprintf(f, "%d %d %d %d %d %d %.6f\n", kv.first.order, kv.first.nx, kv.first.ny, kv.first.nz, kv.first.bc,
                 kv.second.first, kv.second.second);
  const bool bad = std::ferror(f) != 0;
  std::fclose(f);
  return bad ? PN_ERR_ARG : PN_OK;
}

extern "C" pn_status pn_tune_cache_load(const char* path) {
  if (!path) return PN_ERR_ARG;
  FILE* f = std::fopen(path, "r");
  if (!f) return PN_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  char line[256];
  pn_status st = PN_OK;
  while (std::fgets(line, sizeof(line), f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    TuneKey k{};
    int z = 0;
    double ms = 0.0;
    if (std::sscanf(line, "%d %d %d %d %d %d %lf", &k.order, &k.nx, &k.ny, &k.nz, &k.bc, &z, &ms) != 7 ||
        k.order < 1 || k.order > PN_MAX_ORDER || k.nx < 1 || k.ny < 1 || k.nz < 1 || z < 1 ||
        k.bc < 0 || k.bc >= 27) {
      st = PN_ERR_ARG;
      break;
    }
    g_tune[k] = {z, ms};
  }
  std::fclose(f);
  return st;
}

pn_status setup_ctx(int order, const pn_grid* grid, const pn_medium* med, void* stream, bool workspace,
                    pn_ctx** out) {
  pn_ctx* c = nullptr;
  if (!out) return fail(nullptr, PN_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (order < 1 || order > PN_MAX_ORDER) return fail(nullptr, PN_ERR_ARG, "order must be in 1..7");
  if (!grid || !med) return fail(nullptr, PN_ERR_ARG, "grid or medium is NULL");
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return fail(nullptr, PN_ERR_ARG, "grid dimensions must be >= 1");
  int bcs[3];
  for (int d = 0; d < 3; ++d) bcs[d] = grid->bc == PN_BC_PER_AXIS ? grid->bc_axis[d] : grid->bc;
  for (int d = 0; d < 3; ++d)
    if (bcs[d] != PN_BC_VACUUM && bcs[d] != PN_BC_PERIODIC && bcs[d] != PN_BC_NEUMANN)
      return fail(nullptr, PN_ERR_ARG, "unknown boundary type");
  if (!med->sigma_t || !med->albedo) return fail(nullptr, PN_ERR_ARG, "medium arrays are NULL");
  if (!(med->g > -1.f && med->g < 1.f)) return fail(nullptr, PN_ERR_ARG, "g must be in (-1, 1)");
  if (!(med->sigma_t_min >= 0.f) || !std::isfinite(med->sigma_t_min)) return fail(nullptr, PN_ERR_ARG, "sigma_t_min must be finite and >= 0");
  const long cells = (long)grid->nx * grid->ny * grid->nz;
  if (cells > (1L << 30)) return fail(nullptr, PN_ERR_ARG, "grid too large");

  c = new pn_ctx();
  c->order = order;
  c->nc = (order + 1) * (order + 1);
  c->nx = grid->nx; c->ny = grid->ny; c->nz = grid->nz; c->bc = grid->bc;
  for (int d = 0; d < 3; ++d) c->bcs[d] = bcs[d];
  c->h = grid->h > 0.0 ? grid->h : 1.0 / grid->nx;
  c->g = med->g;
  c->thr = med->sigma_t_min;
  c->stream = (hipStream_t)stream;
  long n = 0;
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
      c->ext[k][d] = dims[d] + (c->bcs[d] == BC_PERIODIC ? 0 : p[d]);
      sz *= c->ext[k][d];
    }
    c->off[k] = (int)n;
    n += sz;
    if (n >= (1L << 31) - 1) { delete c; return fail(nullptr, PN_ERR_ARG, "too many unknowns (>= 2^31)"); }
  }
  c->n = n;
  c->even.nk = 0;
  for (int k = 0; k < c->nc; ++k) {
    int l = 0;
    while ((l + 1) * (l + 1) <= k) ++l;
    if ((l & 1) == 0) c->even.k[c->even.nk++] = k;
  }
  set_geometry(c, 0);
  c->max_blocks = 1 << 16;
  if (c->nblocks > c->max_blocks) { delete c; return fail(nullptr, PN_ERR_ARG, "grid too large in x*y"); }
  if (c->nv >= (1LL << 31) - 1) {  // kernels use 32-bit element offsets
    delete c;
    return fail(nullptr, PN_ERR_ARG, "too many unknowns for the padded layout (>= 2^31)");
  }

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
  const long long pcells = (long long)(c->nx + 2) * (c->ny + 2) * (c->nz + 2);
  SETUP_HIP(hipMalloc(&c->med, sizeof(float2) * pcells));
  SETUP_HIP(hipMalloc(&c->med32, sizeof(float2) * pcells));
  if (workspace) {
    float** v32[] = {&c->r32[0], &c->r32[1], &c->s32, &c->p32, &c->q32, &c->d32, &c->b32};
    for (float** v : v32) {
      SETUP_HIP(hipMalloc(v, sizeof(float) * c->nv));
      SETUP_HIP(hipMemsetAsync(*v, 0, sizeof(float) * c->nv, c->stream));  // zero halo invariant
    }
    SETUP_HIP(hipMalloc(&c->m16, sizeof(uint16_t) * c->nv));
    SETUP_HIP(hipMemsetAsync(c->m16, 0, sizeof(uint16_t) * c->nv, c->stream));
    SETUP_HIP(hipMalloc(&c->x64, sizeof(double) * c->nv));
    SETUP_HIP(hipMemsetAsync(c->x64, 0, sizeof(double) * c->nv, c->stream));
    SETUP_HIP(hipMalloc(&c->st, sizeof(DevState)));
    SETUP_HIP(hipHostMalloc(&c->st_host, sizeof(DevState), hipHostMallocDefault));
    SETUP_HIP(hipMalloc(&c->partials, sizeof(double) * 2 * c->max_blocks));
  }
  SETUP_HIP(hipMalloc(&c->flag, sizeof(int)));
  SETUP_HIP(hipHostMalloc(&c->flag_host, sizeof(int), hipHostMallocDefault));

  SETUP_HIP(hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
  hipLaunchKernelGGL(k_medium_prep, dim3(grid_for(pcells)), dim3(kBlock), 0, c->stream, med->sigma_t,
                     med->albedo, c->thr, c->nx, c->ny, c->nz, c->bcs[0] == BC_PERIODIC, c->bcs[1] == BC_PERIODIC,
                     c->bcs[2] == BC_PERIODIC, c->med32, c->med, c->flag);
  SETUP_HIP(hipGetLastError());
  SETUP_HIP(hipMemcpyAsync(c->flag_host, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  SETUP_HIP(hipStreamSynchronize(c->stream));
  if (*c->flag_host & 1) return bail(PN_ERR_NONFINITE, "medium contains NaN or Inf");
  c->zero_ext = (*c->flag_host & 2) != 0;
  {
    // LDS per block: 64 KiB by default; up to the device's opt-in limit when
    // the kernel attribute can be raised.
    int dev = 0, optin = 0;
    c->lds_max = 64 * 1024 - 1024;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess &&
        optin > 64 * 1024) {
      const size_t want = std::min<size_t>(kLdsMax, (size_t)optin) - 1024;
      if (lds_prepare_order(c->order, want) == hipSuccess) c->lds_max = want;
      else (void)hipGetLastError();  // clear; keep the default limit
    }
    (void)hipGetLastError();
  }
  choose_tiles(c);
#undef SETUP_HIP
  {
    int z = 0;
    if (tune_lookup(c, &z, nullptr)) set_geometry(c, z);
  }
  *out = c;
  return PN_OK;
}

extern "C" pn_status pn_setup(int order, const pn_grid* grid, const pn_medium* med, void* stream,
                              pn_ctx** out) {
  return setup_ctx(order, grid, med, stream, true, out);
}

void free_ctx(pn_ctx* c) {
  if (!c) return;
  free_all(c);
  delete c;
}

extern "C" pn_status pn_set_zchunk(pn_ctx* c, int zchunk) {
  if (!c) return PN_ERR_ARG;
  if (!c->p32) return fail(c, PN_ERR_ARG, "context has no Krylov workspace (a batch problem context)");
  if (zchunk < 0) return fail(c, PN_ERR_ARG, "zchunk must be >= 0");
  set_geometry(c, zchunk);
  if (c->nblocks > c->max_blocks) { set_geometry(c, 0); return fail(c, PN_ERR_ARG, "too many blocks"); }
  if (c->gexec32) { hipGraphExecDestroy(c->gexec32); c->gexec32 = nullptr; c->giters32 = 0; }
  if (c->gexec64) { hipGraphExecDestroy(c->gexec64); c->gexec64 = nullptr; c->giters64 = 0; }
  if (c->gexec_cg) { hipGraphExecDestroy(c->gexec_cg); c->gexec_cg = nullptr; c->giters_cg = 0; }
  if (c->gexec_schur) { hipGraphExecDestroy(c->gexec_schur); c->gexec_schur = nullptr; c->giters_schur = 0; }
  if (c->gexec_mg) { hipGraphExecDestroy(c->gexec_mg); c->gexec_mg = nullptr; c->giters_mg = 0; }
  return PN_OK;
}

extern "C" pn_status pn_set_tiles(pn_ctx* c, int tx, int ty, int zchunk) {
  if (!c) return PN_ERR_ARG;
  if (!c->p32) return fail(c, PN_ERR_ARG, "context has no Krylov workspace (a batch problem context)");
  if (c->gexec_cg) { hipGraphExecDestroy(c->gexec_cg); c->gexec_cg = nullptr; c->giters_cg = 0; }
  if (c->gexec_schur) { hipGraphExecDestroy(c->gexec_schur); c->gexec_schur = nullptr; c->giters_schur = 0; }
  if (c->gexec_mg) { hipGraphExecDestroy(c->gexec_mg); c->gexec_mg = nullptr; c->giters_mg = 0; }
  if (tx == 0 && ty == 0) {  // back to the register-window stencil
    c->use_lds = 0;
    return PN_OK;
  }
  if (!c->lds_ok) return fail(c, PN_ERR_ARG, "the LDS-tiled stencil is not available for this context");
  const int otx = c->TX, oty = c->TY, oz = c->lzchunk;
  if (!set_tiles(c, tx, ty, zchunk)) {
    set_tiles(c, otx, oty, oz);
    return fail(c, PN_ERR_ARG, "tile shape not usable");
  }
  c->use_lds = 1;
  return PN_OK;
}

extern "C" pn_status pn_get_tiles(const pn_ctx* c, int* tx, int* ty, int* zchunk) {
  if (!c || !tx || !ty || !zchunk) return PN_ERR_ARG;
  *tx = c->use_lds ? c->TX : 0;
  *ty = c->use_lds ? c->TY : 0;
  *zchunk = c->use_lds ? c->lzchunk : c->zchunk;
  return PN_OK;
}

extern "C" int pn_get_zchunk(const pn_ctx* c) { return c ? c->zchunk : -1; }

extern "C" pn_status pn_layout_query(const pn_ctx* c, pn_layout* L) {
  if (!c || !L) return PN_ERR_ARG;
  std::memset(L, 0, sizeof(*L));
  L->order = c->order; L->ncoeff = c->nc;
  L->nx = c->nx; L->ny = c->ny; L->nz = c->nz; L->bc = c->bc;
  for (int d = 0; d < 3; ++d) L->bc_axis[d] = c->bcs[d];
  L->n_unknowns = c->n;
  for (int k = 0; k < c->nc; ++k) {
    for (int d = 0; d < 3; ++d) { L->cls[k][d] = c->cls[k][d]; L->ext[k][d] = c->ext[k][d]; }
    L->offset[k] = c->off[k];
  }
  L->offset[c->nc] = c->n;
  return PN_OK;
}

static pn_status ensure64(pn_ctx* c) {
  if (c->s64) return PN_OK;
  double** v[] = {&c->r64[0], &c->r64[1], &c->s64, &c->p64, &c->q64, &c->d64};
  for (double** p : v) {
    PN_HIP(hipMalloc(p, sizeof(double) * c->nv));
    PN_HIP(hipMemsetAsync(*p, 0, sizeof(double) * c->nv, c->stream));
  }
  return PN_OK;
}

extern "C" pn_status pn_apply(pn_ctx* c, const float* x, float* y, int transpose) {
  if (!c) return PN_ERR_ARG;
  if (!c->p32) return fail(c, PN_ERR_ARG, "context has no Krylov workspace (a batch problem context)");
  if (!x || !y) return fail(c, PN_ERR_ARG, "x or y is NULL");
  if ((const void*)x == (const void*)y) return fail(c, PN_ERR_ARG, "x and y must not alias");
  // packed -> padded (p32), apply into q32, padded -> packed
  PN_HIP((launch_pack<float, float, 0>(c, x, c->p32, c->stream)));
  StencilArgs a = base_args(c);
  a.tsign = transpose ? -1.0 : 1.0;
  a.x = c->p32; a.y = c->q32;
  if (c->use_lds) PN_HIP(launch_lds(c, M_APPLY, false, a, c->stream));
  else PN_HIP((launch_stencil<float, M_APPLY, float>(c, a, c->stream)));
  PN_HIP((launch_pack<float, float, 1>(c, c->q32, y, c->stream)));
  return PN_OK;
}

static bool schur_ok(const pn_ctx* c);
static int pcg_vec_blocks(const pn_ctx* c);
static bool mg_ok(const pn_ctx* c);
static pn_status schur_prepare(pn_ctx* c, bool mg, hipStream_t st);
static hipError_t mg_vcycle(pn_ctx* c, const float* r, hipStream_t st);
static const float* mg_final(const pn_ctx* c, int L);
constexpr float kMgOmegaFine = 0.6f;  // weight of the Jacobi part of B

static RenderArgs render_args(const pn_ctx* c) {
  RenderArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nc = c->nc; a.nx = c->nx; a.ny = c->ny; a.nz = c->nz;
  for (int d = 0; d < 3; ++d) a.per[d] = c->bcs[d] == BC_PERIODIC;
  for (int k = 0; k < c->nc; ++k) {
    a.off[k] = c->off[k];
    for (int d = 0; d < 3; ++d) { a.ext[k][d] = c->ext[k][d]; a.cls[k][d] = c->cls[k][d]; }
  }
  a.h = c->h;
  a.g = (double)c->g;
  a.med = c->med;
  return a;
}

static int render_grid(long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  return (int)std::max<long long>(1, std::min<long long>(b, 4096));
}

extern "C" pn_status pn_single_scatter(pn_ctx* c, const double* light, double power, float* rhs) {
  if (!c) return PN_ERR_ARG;
  if (!light || !rhs) return fail(c, PN_ERR_ARG, "light or rhs is NULL");
  if (!std::isfinite(light[0]) || !std::isfinite(light[1]) || !std::isfinite(light[2]) || !std::isfinite(power))
    return fail(c, PN_ERR_ARG, "light position and power must be finite");
  if (c->bcs[0] == BC_PERIODIC || c->bcs[1] == BC_PERIODIC || c->bcs[2] == BC_PERIODIC)
    return fail(c, PN_ERR_ARG, "single scattering needs a non-periodic domain");
  RenderArgs a = render_args(c);
  for (int d = 0; d < 3; ++d) a.light[d] = light[d];
  a.power = power;
  long long maxsz = 0;
  for (int k = 0; k < c->nc; ++k) maxsz = std::max<long long>(maxsz, (long long)c->ext[k][0] * c->ext[k][1] * c->ext[k][2]);
  hipLaunchKernelGGL(k_single_scatter, dim3(render_grid(maxsz), c->nc), dim3(kBlock), 0, c->stream, a, rhs);
  PN_HIP(hipGetLastError());
  return PN_OK;
}

extern "C" pn_status pn_unstagger(pn_ctx* c, const double* x, float* out) {
  if (!c) return PN_ERR_ARG;
  if (!x || !out) return fail(c, PN_ERR_ARG, "x or out is NULL");
  const RenderArgs a = render_args(c);
  const long long cells = (long long)c->nx * c->ny * c->nz;
  hipLaunchKernelGGL(k_unstagger, dim3(render_grid(cells), c->nc), dim3(kBlock), 0, c->stream, a, x, out);
  PN_HIP(hipGetLastError());
  return PN_OK;
}

extern "C" pn_status pn_apply_schur(pn_ctx* c, const float* x, float* y) {
  if (!c) return PN_ERR_ARG;
  if (!c->p32) return fail(c, PN_ERR_ARG, "context has no Krylov workspace (a batch problem context)");
  if (!x || !y) return fail(c, PN_ERR_ARG, "x or y is NULL");
  if ((const void*)x == (const void*)y) return fail(c, PN_ERR_ARG, "x and y must not alias");
  if (!schur_ok(c)) return fail(c, PN_ERR_ARG, "the even-parity operator needs T_oe = -T_eo^T (no Neumann axis) and positive extinction in every cell");
  PN_HIP((launch_pack<float, float, 0>(c, x, c->p32, c->stream)));
  StencilArgs a = base_args(c);
  a.partials = c->partials;
  a.x = c->p32; a.y = c->p32;  // odd slots of p32 <- -D_o^-1 T_oe x_e
  PN_HIP((launch_stencil<float, M_ODD_W, float>(c, a, c->stream)));
  a.x = c->p32; a.y = c->q32;
  PN_HIP((launch_stencil<float, M_EVEN_S, float>(c, a, c->stream)));
  // y: even bands from q32, odd bands from p32
  PN_HIP((launch_pack<float, float, 1>(c, c->q32, y, c->stream)));
  PackArgs pa = pack_args(c);
  for (int k = 0; k < c->nc; ++k) {
    int l = 0;
    while ((l + 1) * (l + 1) <= k) ++l;
    if ((l & 1) == 0) pa.ex[k] = 0;  // even bands: keep what came from q32
  }
  PN_HIP((launch_pack_args<float, float, 1>(c, pa, c->p32, y, c->stream)));
  return PN_OK;
}

extern "C" pn_status pn_apply_precond(pn_ctx* c, int variant, const float* r, float* z) {
  if (!c) return PN_ERR_ARG;
  if (!c->p32) return fail(c, PN_ERR_ARG, "context has no Krylov workspace (a batch problem context)");
  if (!r || !z) return fail(c, PN_ERR_ARG, "r or z is NULL");
  if ((const void*)r == (const void*)z) return fail(c, PN_ERR_ARG, "r and z must not alias");
  if (variant != PN_VARIANT_SCHUR && variant != PN_VARIANT_SCHUR_MG)
    return fail(c, PN_ERR_ARG, "variant must be PN_VARIANT_SCHUR or PN_VARIANT_SCHUR_MG");
  const bool mg = variant == PN_VARIANT_SCHUR_MG;
  if (!schur_ok(c)) return fail(c, PN_ERR_ARG, "the even-parity preconditioner needs no Neumann axis and positive extinction");
  if (mg && !mg_ok(c)) return fail(c, PN_ERR_ARG, "the multigrid preconditioner needs no Neumann axis and positive extinction");
  const int need = mg ? 3 : 1;
  if ((c->prec_ready & need) != need) {
    pn_status e = schur_prepare(c, mg, c->stream);
    if (e != PN_OK) return e;
  }
  DevState init;
  std::memset(&init, 0, sizeof(init));
  PN_HIP(hipMemcpyAsync(c->st, &init, sizeof(DevState), hipMemcpyHostToDevice, c->stream));
  PN_HIP((launch_pack<float, float, 0>(c, r, c->r32[1], c->stream)));
  hipLaunchKernelGGL((k_fill<float>), dim3(grid_for(c->nv)), dim3(kBlock), 0, c->stream, c->p32, (long)c->nv, 0.f);
  PN_HIP(hipGetLastError());
  const dim3 vg(pcg_vec_blocks(c), c->even.nk);
  if (mg) {
    PN_HIP(mg_vcycle(c, c->r32[1], c->stream));
    hipLaunchKernelGGL(k_pcg_vec_mg<4>, vg, dim3(kBlock), 0, c->stream, c->d32, (const float*)c->r32[1], c->p32,
                       (const uint16_t*)c->m16, c->mg_fine, c->mg_geom[1], mg_final(c, 1), kMgOmegaFine,
                       (const DevState*)c->st);
  } else {
    hipLaunchKernelGGL(k_pcg_vec<0>, vg, dim3(kBlock), 0, c->stream, c->d32, c->r32[1], c->p32, (const float*)c->q32,
                       (const uint16_t*)c->m16, c->even, c->partials, (const DevState*)c->st);
  }
  PN_HIP(hipGetLastError());
  PN_HIP((launch_pack<float, float, 1>(c, c->p32, z, c->stream)));
  return PN_OK;
}

extern "C" pn_status pn_row_weights(pn_ctx* c, float* w) {
  if (!c) return PN_ERR_ARG;
  if (!c->p32) return fail(c, PN_ERR_ARG, "context has no Krylov workspace (a batch problem context)");
  if (!w) return fail(c, PN_ERR_ARG, "w is NULL");
  // W applied to the all-ones vector
  hipLaunchKernelGGL((k_fill<float>), dim3(grid_for(c->n)), dim3(kBlock), 0, c->stream, w, (long)c->n, 1.0f);
  PN_HIP(hipGetLastError());
  PN_HIP((launch_pack<float, float, 0>(c, w, c->p32, c->stream)));
  StencilArgs a = base_args(c);
  a.x = c->p32; a.y = c->q32; a.partials = c->partials;
  PN_HIP((launch_stencil<float, M_EQS, float>(c, a, c->stream)));
  PN_HIP((launch_pack<float, float, 1>(c, c->q32, w, c->stream)));
  return PN_OK;
}

extern "C" pn_status pn_apply64(pn_ctx* c, const double* x, double* y, int transpose) {
  if (!c) return PN_ERR_ARG;
  if (!c->p32) return fail(c, PN_ERR_ARG, "context has no Krylov workspace (a batch problem context)");
  if (!x || !y) return fail(c, PN_ERR_ARG, "x or y is NULL");
  if ((const void*)x == (const void*)y) return fail(c, PN_ERR_ARG, "x and y must not alias");
  pn_status e = ensure64(c);
  if (e != PN_OK) return e;
  PN_HIP((launch_pack<double, double, 0>(c, x, c->p64, c->stream)));
  StencilArgs a = base_args(c);
  a.tsign = transpose ? -1.0 : 1.0;
  a.x = c->p64; a.y = c->q64;
  PN_HIP((launch_stencil<double, M_APPLY, double>(c, a, c->stream)));
  PN_HIP((launch_pack<double, double, 1>(c, c->q64, y, c->stream)));
  return PN_OK;
}

// Times `iters` back-to-back FP32 applies on the padded workspace (the apply
// of the Krylov loop) with HIP events on the context stream.
extern "C" pn_status pn_bench_apply(pn_ctx* c, int iters, int transpose, double* ms_per_apply) {
  if (!c || iters < 1 || !ms_per_apply) return c ? fail(c, PN_ERR_ARG, "bad arguments") : PN_ERR_ARG;
  if (!c->p32) return fail(c, PN_ERR_ARG, "context has no Krylov workspace (a batch problem context)");
  hipEvent_t e0, e1;
  PN_HIP(hipEventCreate(&e0));
  PN_HIP(hipEventCreate(&e1));
  StencilArgs a = base_args(c);
  a.tsign = transpose ? -1.0 : 1.0;
  a.x = c->p32; a.y = c->q32;
  auto one = [&]() -> hipError_t {
    return c->use_lds ? launch_lds(c, M_APPLY, false, a, c->stream)
                     : launch_stencil<float, M_APPLY, float>(c, a, c->stream);
  };
  PN_HIP(one());  // warm-up
  PN_HIP(hipEventRecord(e0, c->stream));
  for (int i = 0; i < iters; ++i) PN_HIP(one());
  PN_HIP(hipEventRecord(e1, c->stream));
  PN_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  PN_HIP(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *ms_per_apply = ms / iters;
  return PN_OK;
}

// Times one kernel of the FP32 Krylov loop with HIP events on the context
// stream.  The plain applies run `iters` times back to back.  The in-loop
// kernels run inside `iters` iterations of the loop's own sequence
// (q = W A p, s -= alpha A^T q, x/p update), so each sees the cache state it
// sees in a solve; events around the requested kernel give its mean time.
// The device scalars are reset first (alpha = beta = 0.5, no stop flag); the
// next solve re-initialises them.


extern "C" pn_status pn_bench_kernel(pn_ctx* c, int kernel, int iters, double* ms) {
  if (!c || iters < 1 || !ms || kernel < PN_KERNEL_APPLY || kernel > PN_KERNEL_PCG_XP_MG)
    return c ? fail(c, PN_ERR_ARG, "bad arguments") : PN_ERR_ARG;
  if (!c->p32) return fail(c, PN_ERR_ARG, "context has no Krylov workspace (a batch problem context)");
  if (c->use_lds && kernel != PN_KERNEL_APPLY && kernel != PN_KERNEL_APPLY_T)
    return fail(c, PN_ERR_ARG, "the in-loop kernels are timed on the register-window stencil");
  const bool mgk = kernel >= PN_KERNEL_MG_VCYCLE;
  if (mgk) {
    if (!mg_ok(c)) return fail(c, PN_ERR_ARG, "the multigrid kernels need no Neumann axis and positive extinction");
    pn_status e = schur_prepare(c, true, c->stream);  // Jacobi diagonal and multigrid operators
    if (e != PN_OK) return e;
  }
  DevState init;
  std::memset(&init, 0, sizeof(init));
  init.alpha = 0.5;
  init.beta = 0.5;
  PN_HIP(hipMemcpyAsync(c->st, &init, sizeof(DevState), hipMemcpyHostToDevice, c->stream));
  hipEvent_t e0, e1;
  PN_HIP(hipEventCreate(&e0));
  PN_HIP(hipEventCreate(&e1));
  auto launch = [&](int k) -> hipError_t {
    StencilArgs a = base_args(c);
    switch (k) {
      case PN_KERNEL_APPLY:
      case PN_KERNEL_APPLY_T:
        a.tsign = k == PN_KERNEL_APPLY_T ? -1.0 : 1.0;
        a.x = c->p32; a.y = c->q32;
        return c->use_lds ? launch_lds(c, M_APPLY, false, a, c->stream)
                          : launch_stencil<float, M_APPLY, float>(c, a, c->stream);
      case PN_KERNEL_APPLY_EQ:
        a.st = c->st; a.partials = c->partials; a.tsign = 1.0;
        a.x = c->p32; a.y = c->q32;
        return launch_stencil<float, M_APPLY_EQ, float>(c, a, c->stream);
      case PN_KERNEL_SUPD:
        a.st = c->st; a.partials = c->partials; a.tsign = -1.0;
        a.x = c->q32; a.y = c->s32;
        return launch_stencil<float, M_SUPD, float>(c, a, c->stream);
      case PN_KERNEL_ODD_W:
        a.st = c->st; a.partials = c->partials; a.x = c->p32; a.y = c->p32;
        return launch_stencil<float, M_ODD_W, float>(c, a, c->stream);
      case PN_KERNEL_EVEN_R:
        a.st = c->st; a.partials = c->partials; a.x = c->p32; a.y = c->r32[1]; a.m16 = c->m16;
        return launch_stencil<float, M_EVEN_SR, float>(c, a, c->stream);
      case PN_KERNEL_PCG_XP: {
        const dim3 vg(pcg_vec_blocks(c), c->even.nk);
        hipLaunchKernelGGL(k_pcg_vec<2>, vg, dim3(kBlock), 0, c->stream, c->d32, c->r32[1], c->p32,
                           (const float*)c->q32, (const uint16_t*)c->m16, c->even, c->partials, (const DevState*)c->st);
        return hipGetLastError();
      }
      case PN_KERNEL_MG_VCYCLE:
        return mg_vcycle(c, c->r32[1], c->stream);
      case PN_KERNEL_PCG_XP_MG: {
        const dim3 vg(pcg_vec_blocks(c), c->even.nk);
        hipLaunchKernelGGL(k_pcg_vec_mg<2>, vg, dim3(kBlock), 0, c->stream, c->d32, (const float*)c->r32[1], c->p32,
                           (const uint16_t*)c->m16, c->mg_fine, c->mg_geom[1], mg_final(c, 1), kMgOmegaFine,
                           (const DevState*)c->st);
        return hipGetLastError();
      }
      default:
        hipLaunchKernelGGL((k_update_xp<float>), dim3(stream_grid(c->nv / 4)), dim3(kBlock), 0, c->stream, c->d32,
                           c->p32, (const float*)c->s32, (long)c->nv, (const DevState*)c->st);
        return hipGetLastError();
    }
  };
  double total = 0.0;
  if (kernel == PN_KERNEL_APPLY || kernel == PN_KERNEL_APPLY_T) {
    PN_HIP(launch(kernel));  // warm-up
    PN_HIP(hipEventRecord(e0, c->stream));
    for (int i = 0; i < iters; ++i) PN_HIP(launch(kernel));
    PN_HIP(hipEventRecord(e1, c->stream));
    PN_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    PN_HIP(hipEventElapsedTime(&t, e0, e1));
    total = t;
  } else {
    const int seq_cg[4] = {PN_KERNEL_APPLY_EQ, PN_KERNEL_SUPD, PN_KERNEL_UPDATE, -1};
    const int seq_schur[4] = {PN_KERNEL_ODD_W, PN_KERNEL_EVEN_R, PN_KERNEL_PCG_XP, -1};
    const int seq_mg[4] = {PN_KERNEL_ODD_W, PN_KERNEL_EVEN_R, PN_KERNEL_MG_VCYCLE, PN_KERNEL_PCG_XP_MG};
    const int* seq = mgk ? seq_mg : (kernel >= PN_KERNEL_ODD_W ? seq_schur : seq_cg);
    for (int i = 0; i <= iters; ++i) {  // iteration 0 warms up
      for (int j = 0; j < 4; ++j) {
        const int k = seq[j];
        if (k < 0) break;
        if (k == kernel) PN_HIP(hipEventRecord(e0, c->stream));
        PN_HIP(launch(k));
        if (k == kernel) PN_HIP(hipEventRecord(e1, c->stream));
      }
      PN_HIP(hipEventSynchronize(e1));
      float t = 0.f;
      PN_HIP(hipEventElapsedTime(&t, e0, e1));
      if (i > 0) total += t;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *ms = total / iters;
  return PN_OK;
}

// r = Q - A x in FP64 arithmetic on padded vectors; partials -> st->rtrue2, st->bb2.
template <typename TO>
static pn_status residual(pn_ctx* c, const float* rhs_pad, const double* x_pad, TO* r_pad, hipStream_t s) {
  StencilArgs a = base_args(c);
  a.x = x_pad; a.x2 = rhs_pad; a.y = r_pad;
  a.partials = c->partials;
  PN_HIP((launch_stencil<double, M_RESID, TO>(c, a, s)));
  hipLaunchKernelGGL(k_fin_resid, dim3(1), dim3(kFinBlock), 0, s, c->st, c->partials, c->nblocks);
  PN_HIP(hipGetLastError());
  return PN_OK;
}

extern "C" pn_status pn_residual64(pn_ctx* c, const float* rhs, const double* x, double* r, double* rel) {
  if (!c) return PN_ERR_ARG;
  if (!c->p32) return fail(c, PN_ERR_ARG, "context has no Krylov workspace (a batch problem context)");
  if (!rhs || !x) return fail(c, PN_ERR_ARG, "rhs or x is NULL");
  pn_status s = ensure64(c);
  if (s != PN_OK) return s;
  PN_HIP((launch_pack<float, float, 0>(c, rhs, c->b32, c->stream)));
  PN_HIP((launch_pack<double, double, 0>(c, x, c->x64, c->stream)));
  s = residual<double>(c, c->b32, c->x64, c->r64[0], c->stream);
  if (s != PN_OK) return s;
  if (r) PN_HIP((launch_pack<double, double, 1>(c, c->r64[0], r, c->stream)));
  PN_HIP(hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
  PN_HIP(hipStreamSynchronize(c->stream));
  if (rel) *rel = c->st_host->bb2 > 0.0 ? std::sqrt(c->st_host->rtrue2 / c->st_host->bb2) : 0.0;
  return PN_OK;
}

// One CGLS iteration on padded vectors of type T (r ping-pong rin -> rout).
template <typename T>
static hipError_t enqueue_iteration(pn_ctx* c, T* d, T* p, T* q, T* s, const T* rin, T* rout, hipStream_t st) {
  StencilArgs a = base_args(c);
  a.st = c->st;
  a.partials = c->partials;
  a.x = p; a.y = q; a.tsign = 1.0;
  hipError_t e = launch_stencil<T, M_APPLY, T>(c, a, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(kFinBlock), 0, st, c->st, c->partials, c->nblocks);
  a.x = rin; a.x2 = q; a.y = s; a.y2 = rout; a.tsign = -1.0;
  e = launch_stencil<T, M_TRANSR, T>(c, a, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fin_beta, dim3(1), dim3(kFinBlock), 0, st, c->st, c->partials, c->nblocks);
  hipLaunchKernelGGL((k_update_xp<T>), dim3(stream_grid(c->nv / (sizeof(T) == 4 ? 4 : 1))), dim3(kBlock), 0, st,
                     d, p, (const T*)s, (long)c->nv, (const DevState*)c->st);
  return hipGetLastError();
}

// One iteration of CG on the normal equations (FP32 vectors; LDS-tiled or
// register-window stencil):
// q = A p | alpha | s -= alpha A^T q | beta | x += alpha p, p = s + beta p.
// Row-equilibrated (eq, register-window stencil only): CG on A^T W A u = A^T W r
// with W = diag(1 / ||row of A||^2): q = W A p, alpha = gamma / <A p, W A p>,
// the rest unchanged.
static hipError_t enqueue_iteration_cg(pn_ctx* c, float* d, float* p, float* q, float* s, bool eq, hipStream_t st) {
  StencilArgs a = base_args(c);
  a.st = c->st;
  a.partials = c->partials;
  a.x = p; a.y = q; a.tsign = 1.0;
  const int nb = c->use_lds ? c->lnblocks : c->nblocks;
  hipError_t e = c->use_lds ? launch_lds(c, M_APPLY, true, a, st)
                 : eq       ? launch_stencil<float, M_APPLY_EQ, float>(c, a, st)
                            : launch_stencil<float, M_APPLY, float>(c, a, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fin_alpha_cg, dim3(1), dim3(kFinBlock), 0, st, c->st, c->partials, nb);
  a.x = q; a.y = s; a.tsign = -1.0;
  e = c->use_lds ? launch_lds(c, M_SUPD, true, a, st) : launch_stencil<float, M_SUPD, float>(c, a, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fin_beta_cg, dim3(1), dim3(kFinBlock), 0, st, c->st, c->partials, nb);
  hipLaunchKernelGGL((k_update_xp<float>), dim3(stream_grid(c->nv / 4)), dim3(kBlock), 0, st, d, p,
                     (const float*)s, (long)c->nv, (const DevState*)c->st);
  return hipGetLastError();
}

// Even-parity PCG (Schur complement S = D_e - T_eo D_o^-1 T_oe, Jacobi
// preconditioner m = 1 / diag(S) in the even slots of s32; PCG vectors in the
// even slots: x = d32, r = r32[1], p = p32, q = q32):
// w_o = -D_o^-1 T_oe p_e (odd slots of p) | q_e = S p_e | alpha | x, r update |
// beta | p = m r + beta p.
static int pcg_vec_blocks(const pn_ctx* c) {
  const long long n4 = c->cs / 4;
  const long long b = (n4 + kBlock - 1) / kBlock;
  return (int)std::max<long long>(1, std::min<long long>(b, 256));
}

static hipError_t enqueue_iteration_schur(pn_ctx* c, hipStream_t st) {
  StencilArgs a = base_args(c);
  a.st = c->st;
  a.tsign = 1.0;
  a.partials = c->partials;
  // w_o = -D_o^-1 T_oe p_e with the partials of <p, S p> = <p_e, D_e p_e> + <w_o, D_o w_o>
  a.x = c->p32; a.y = c->p32;
  hipError_t e = launch_stencil<float, M_ODD_W, float>(c, a, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fin_alpha_pcg, dim3(1), dim3(kFinBlock), 0, st, c->st, c->partials, c->nblocks);
  // r -= alpha (D_e p_e + T_eo w_o) with the partials of <r, M r>, <r, r>
  a.x = c->p32; a.y = c->r32[1]; a.m16 = c->m16;
  e = launch_stencil<float, M_EVEN_SR, float>(c, a, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fin_beta_pcg, dim3(1), dim3(kFinBlock), 0, st, c->st, c->partials, c->nblocks);
  const dim3 vg(pcg_vec_blocks(c), c->even.nk);
  hipLaunchKernelGGL(k_pcg_vec<2>, vg, dim3(kBlock), 0, st, c->d32, c->r32[1], c->p32, (const float*)c->q32,
                     (const uint16_t*)c->m16, c->even, c->partials, (const DevState*)c->st);
  return hipGetLastError();
}

static pn_status build_graph_schur(pn_ctx* c, int iters, hipGraphExec_t* exec) {
  hipGraph_t g = nullptr;
  PN_HIP(hipStreamBeginCapture(c->sstream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int i = 0; i < iters && e == hipSuccess; ++i) e = enqueue_iteration_schur(c, c->sstream);
  hipError_t e2 = hipStreamEndCapture(c->sstream, &g);
  if (e != hipSuccess) { if (g) hipGraphDestroy(g); return fail(c, PN_ERR_HIP, std::string("capture: ") + hipGetErrorString(e)); }
  if (e2 != hipSuccess) return fail(c, PN_ERR_HIP, std::string("end capture: ") + hipGetErrorString(e2));
  hipError_t e3 = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e3 != hipSuccess) return fail(c, PN_ERR_HIP, std::string("instantiate: ") + hipGetErrorString(e3));
  return PN_OK;
}

// True when A = [[D_e, T_eo], [T_oe, D_o]] has T_oe = -T_eo^T (no Neumann
// axis) and D_o is invertible (positive extinction everywhere: sigma_t -
// g^l sigma_s > 0 for odd l), so that the even-parity Schur complement
// exists and is symmetric positive definite.
static bool schur_ok(const pn_ctx* c) {
  return c->bcs[0] != BC_NEUMANN && c->bcs[1] != BC_NEUMANN && c->bcs[2] != BC_NEUMANN && !c->zero_ext;
}

// ------------------------------------------------ multigrid preconditioner --
// B r = omega_f M r + P V(P^T r) (see pn_mg.h).  Aggregation runs over the
// class extents; a periodic axis is cut at its seam in the preconditioner
// (the padded halo the coarse operators are formed from holds zeros there, so
// the seam faces' weights stay on the diagonal: B remains symmetric positive
// definite, only less accurate next to the seam).
constexpr float kMgOmega = 0.9f;      // damped Jacobi on the coarse levels
constexpr int kMgSweeps = 16;         // damped Jacobi sweeps on the coarsest level
constexpr int kMgCoarsest = 5;        // coarsen until every axis has at most this many points

static bool mg_ok(const pn_ctx* c) { return schur_ok(c) && c->even.nk >= 1 && c->even.nk <= kMgMaxEven; }

// AUTO's choice of the multigrid form: odd orders (with even N the top band
// stays in the even set and the per-coefficient blocks miss its coupling to
// l = N - 2: 1.0-1.7x fewer iterations against Jacobi, not enough for the
// V-cycle's cost) with at least 2^17 even-band unknowns (below that its
// launches cost more per iteration than the iterations they save).
constexpr long long kMgAutoMinEven = 1LL << 17;
static bool mg_auto(const pn_ctx* c) {
  long long ne = 0;
  for (int s = 0; s < c->even.nk; ++s) {
    const int k = c->even.k[s];
    ne += (long long)c->ext[k][0] * c->ext[k][1] * c->ext[k][2];
  }
  return (c->order & 1) && ne >= kMgAutoMinEven;
}

static long long mg_points(const MgGeom& g, int s) { return (long long)g.ext[s][0] * g.ext[s][1] * g.ext[s][2]; }

static int mg_blocks(const MgGeom& g) {
  long long m = 0;
  for (int s = 0; s < g.nk; ++s) m = std::max(m, mg_points(g, s));
  const long long b = (m + kBlock - 1) / kBlock;
  return (int)std::max<long long>(1, std::min<long long>(b, 2048));
}

// Grid of the aggregating down pass from level f to level c: blocks of
// kBlock / kMgAggLanes aggregates of the largest coarse (x, y) plane, chunks of
// mg_down_chunk coarse z planes of the deepest slot, slots.
static int mg_down_chunk(const MgGeom& f) { return f.off[f.nk] > (1 << 20) ? 2 : 1; }

static dim3 mg_down_grid(const MgGeom& f, const MgGeom& c) {
  long long na = 0;
  int zc = 0;
  for (int s = 0; s < c.nk; ++s) {
    na = std::max(na, (long long)c.ext[s][0] * c.ext[s][1]);
    zc = std::max(zc, c.ext[s][2]);
  }
  const long long b = (na * kMgAggLanes + kBlock - 1) / kBlock;
  const int ch = mg_down_chunk(f);
  return dim3((unsigned)b, (zc + ch - 1) / ch, c.nk);
}

// z planes per thread of the up pass on level f: a march of 4 planes where
// the level has more than 2^20 points (fewer, larger blocks keep z' of the
// plane below in registers), one plane below (more threads in flight).
static int mg_up_chunk(const MgGeom& f) { return f.off[f.nk] > (1 << 20) ? 4 : 1; }

// Grid of the up pass on level f: blocks of the largest (x, y) plane, z
// chunks of the deepest slot, slots.
static dim3 mg_up_grid(const MgGeom& f) {
  long long np = 0;
  int ez = 0;
  for (int s = 0; s < f.nk; ++s) {
    np = std::max(np, (long long)f.ext[s][0] * f.ext[s][1]);
    ez = std::max(ez, f.ext[s][2]);
  }
  const int ch = mg_up_chunk(f);
  return dim3((unsigned)((np + kBlock - 1) / kBlock), (ez + ch - 1) / ch, f.nk);
}

static int mg_restrict_blocks(const MgGeom& g) {
  long long m = 0;
  for (int s = 0; s < g.nk; ++s) m = std::max(m, mg_points(g, s));
  const long long per = (long long)kBlock * kMgRestrictPer;
  return (int)std::max<long long>(1, std::min<long long>((m + per - 1) / per, 2048));
}

// Level geometry, coupling terms and buffers (once per context).
static pn_status mg_alloc(pn_ctx* c) {
  if (c->mg_levels > 0) return PN_OK;
  MgFine& f = c->mg_fine;
  std::memset(&f, 0, sizeof(f));
  f.nk = c->even.nk; f.PX = c->PX; f.PY = c->PY; f.cs = c->cs;
  MgGeom* g = c->mg_geom;
  std::memset(g, 0, sizeof(MgGeom) * kMgMaxLevels);
  g[0].nk = f.nk;
  int slot_of[kMaxCoeff];
  for (int k = 0; k < kMaxCoeff; ++k) slot_of[k] = -1;
  for (int s = 0; s < f.nk; ++s) {
    const int k = c->even.k[s];
    f.k[s] = k;
    slot_of[k] = s;
    for (int d = 0; d < 3; ++d) { f.ext[s][d] = c->ext[k][d]; f.cls[s][d] = c->cls[k][d]; g[0].ext[s][d] = c->ext[k][d]; }
    g[0].off[s + 1] = g[0].off[s] + mg_points(g[0], s);
  }
  int levels = 0;
  for (;;) {
    const MgGeom& a = g[levels];
    MgGeom& b = g[levels + 1];
    b.nk = a.nk;
    int mx = 0;
    for (int s = 0; s < a.nk; ++s) {
      for (int d = 0; d < 3; ++d) { b.ext[s][d] = (a.ext[s][d] + 1) / 2; mx = std::max(mx, b.ext[s][d]); }
      b.off[s + 1] = b.off[s] + mg_points(b, s);
    }
    ++levels;
    if ((mx <= kMgCoarsest && b.off[b.nk] <= kMgCoarseMax) || levels + 1 >= kMgMaxLevels) break;
  }
  if (g[levels].off[g[levels].nk] > kMgCoarseMax) return fail(c, PN_ERR_ARG, "multigrid: coarsest level too large");
  // squared couplings of every even row per axis
  MgTerms t;
  std::memset(&t, 0, sizeof(t));
  const int cap = 8192;
  std::vector<int> tk(cap), td(cap), tkp(cap);
  std::vector<double> tv(cap);
  const int nt = pn_coupling_table(c->order, tk.data(), td.data(), tkp.data(), tv.data(), cap);
  if (nt < 0 || nt > cap) return fail(c, PN_ERR_ARG, "multigrid: coupling table");
  for (int i = 0; i < nt; ++i) {
    const int s = slot_of[tk[i]];
    if (s < 0) continue;
    const int d = td[i];
    int& n = t.n[s][d];
    if (n >= kMgMaxTerms) return fail(c, PN_ERR_ARG, "multigrid: too many couplings of one row along one axis");
    t.j[s][d][n] = tkp[i];
    t.c2[s][d][n] = (float)(tv[i] * tv[i]);
    ++n;
  }
  PN_HIP(hipMalloc(&c->mg_terms, sizeof(MgTerms)));
  PN_HIP(hipMemcpy(c->mg_terms, &t, sizeof(MgTerms), hipMemcpyHostToDevice));
  for (int L = 1; L <= levels; ++L) {
    const size_t n = (size_t)g[L].off[g[L].nk];
    PN_HIP(hipMalloc(&c->mg_op[L], sizeof(float4) * n));
    PN_HIP(hipMalloc(&c->mg_r[L], sizeof(float) * n));
    PN_HIP(hipMalloc(&c->mg_z[L], sizeof(float) * n));
    PN_HIP(hipMalloc(&c->mg_zt[L], sizeof(float) * n));
    PN_HIP(hipMalloc(&c->mg_idg[L], sizeof(float) * n));
  }
  // the tail: the first level L0 < levels at which every slot has at most one
  // point per thread of the tail's block (larger levels keep the wide
  // kernels: one block per slot has too little parallelism there) and its
  // levels L0..levels, plus the scratch, fit the kernel's LDS
  c->mg_tail_L0 = 0;
  for (int L0 = 1; L0 < levels && c->mg_tail_L0 == 0; ++L0) {
    bool fits = true;
    for (int s = 0; s < f.nk && fits; ++s) {
      long long need = mg_points(g[L0 + 1], s);
      for (int L = L0; L <= levels; ++L) need += 2 * mg_points(g[L], s);
      fits = need <= kMgTailLds && mg_points(g[L0], s) <= kFinBlock;
    }
    if (fits) c->mg_tail_L0 = L0;
  }
  if (c->mg_tail_L0 > 0) {
    MgTail tl;
    std::memset(&tl, 0, sizeof(tl));
    tl.L0 = c->mg_tail_L0;
    tl.Lc = levels;
    for (int L = 0; L <= levels; ++L) {
      tl.g[L] = g[L];
      tl.op[L] = c->mg_op[L];
      tl.idg[L] = c->mg_idg[L];
    }
    PN_HIP(hipMalloc(&c->mg_tail, sizeof(MgTail)));
    PN_HIP(hipMemcpy(c->mg_tail, &tl, sizeof(MgTail), hipMemcpyHostToDevice));
  }
  if (levels == 1) {
    c->mg_npart = 1;
  } else if (c->mg_tail_L0 == 1) {
    c->mg_npart = f.nk;
  } else {
    const dim3 gu = mg_up_grid(g[1]);
    c->mg_npart = (int)(gu.x * gu.y * gu.z);
  }
  PN_HIP(hipMalloc(&c->mg_partials, sizeof(double) * 2 * c->mg_npart));
  c->mg_levels = levels;
  return PN_OK;
}

// Operators of every level from the fine diagonal (1 / m32 in the even
// slots) and 1 / d_o (invdo, the odd slots).
static pn_status mg_setup_ops(pn_ctx* c, const float* m32, const float* invdo, hipStream_t st) {
  const MgGeom* g = c->mg_geom;
  hipLaunchKernelGGL(k_mg_setup1, dim3(mg_blocks(g[1]), g[1].nk), dim3(kBlock), 0, st, c->mg_fine, g[1],
                     (const MgTerms*)c->mg_terms, m32, invdo, c->h > 0.0 ? 1.0 / (c->h * c->h) : 0.0, c->mg_op[1],
                     c->mg_idg[1]);
  PN_HIP(hipGetLastError());
  for (int L = 1; L < c->mg_levels; ++L) {
    hipLaunchKernelGGL(k_mg_coarsen, dim3(mg_blocks(g[L + 1]), g[L + 1].nk), dim3(kBlock), 0, st, g[L], g[L + 1],
                       (const float4*)c->mg_op[L], c->mg_op[L + 1], c->mg_idg[L + 1]);
    PN_HIP(hipGetLastError());
  }
  return PN_OK;
}

// Preconditioner setup of the even-parity solve: 1 / d_o in the odd slots of
// q32 (d32 = 0, x2 = NULL reads as 1), m = 1 / diag(S) in the even slots of
// s32 and its bfloat16 copy m16; with `mg`, the multigrid operators.
static pn_status schur_prepare(pn_ctx* c, bool mg, hipStream_t st) {
  hipLaunchKernelGGL((k_fill<float>), dim3(grid_for(c->nv)), dim3(kBlock), 0, st, c->d32, (long)c->nv, 0.f);
  PN_HIP(hipGetLastError());
  StencilArgs a = base_args(c);
  a.x = c->d32; a.x2 = nullptr; a.y = c->q32;
  PN_HIP((launch_stencil<float, M_ODD_BACK, float>(c, a, st)));
  a.x = c->q32; a.y = c->s32;
  PN_HIP((launch_stencil<float, M_EVEN_JAC, float>(c, a, st)));
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(c->nv)), dim3(kBlock), 0, st, (const float*)c->s32, c->m16, (long)c->nv);
  PN_HIP(hipGetLastError());
  c->prec_ready |= 1;
  if (mg) {
    pn_status e = mg_alloc(c);
    if (e == PN_OK) e = mg_setup_ops(c, c->s32, c->q32, st);
    if (e != PN_OK) return e;
    c->prec_ready |= 2;
  }
  return PN_OK;
}

static const float* mg_final(const pn_ctx* c, int L) { return L == c->mg_levels ? c->mg_z[L] : c->mg_zt[L]; }

// One V-cycle on P^T r (fine r: the even slots of the padded r); the level-1
// result in mg_final(c, 1), the partials of <P^T r, V(P^T r)> in mg_partials.
static hipError_t mg_vcycle(pn_ctx* c, const float* r, hipStream_t st) {
  const MgGeom* g = c->mg_geom;
  const int Lc = c->mg_levels;
  const int Lt = c->mg_tail_L0 > 0 ? c->mg_tail_L0 : Lc;  // levels below Lt run one kernel per pass
  const DevState* ds = c->st;
  hipLaunchKernelGGL(k_mg_restrict0, dim3(mg_restrict_blocks(g[1]), g[1].nk), dim3(kBlock), 0, st, c->mg_fine, g[1], r,
                     (const float*)c->mg_idg[1], c->mg_r[1], c->mg_z[1], kMgOmega, ds);
  for (int L = 1; L < Lt; ++L)
    hipLaunchKernelGGL(k_mg_down, mg_down_grid(g[L], g[L + 1]), dim3(kBlock), 0, st, g[L], g[L + 1],
                       (const float4*)c->mg_op[L], (const float*)c->mg_r[L], (const float*)c->mg_z[L],
                       (const float*)c->mg_idg[L + 1], c->mg_r[L + 1], c->mg_z[L + 1], kMgOmega,
                       mg_down_chunk(g[L]), ds);
  if (c->mg_tail_L0 > 0) {
    hipLaunchKernelGGL(k_mg_tail, dim3(g[Lt].nk), dim3(kFinBlock), 0, st, (const MgTail*)c->mg_tail,
                       (const float*)c->mg_r[Lt], (const float*)c->mg_z[Lt], c->mg_zt[Lt], kMgSweeps, kMgOmega,
                       Lt == 1 ? c->mg_partials : (double*)nullptr, ds);
  } else {
    hipLaunchKernelGGL(k_mg_coarsest, dim3(1), dim3(kFinBlock), 0, st, g[Lc], (const float4*)c->mg_op[Lc],
                       (const float*)c->mg_r[Lc], c->mg_z[Lc], kMgSweeps, kMgOmega,
                       Lc == 1 ? c->mg_partials : (double*)nullptr, ds);
  }
  for (int L = Lt - 1; L >= 1; --L)
    hipLaunchKernelGGL(k_mg_up, mg_up_grid(g[L]), dim3(kBlock), 0, st, g[L], g[L + 1],
                       (const float4*)c->mg_op[L], (const float*)c->mg_r[L], (const float*)c->mg_z[L],
                       mg_final(c, L + 1), c->mg_zt[L], kMgOmega, mg_up_chunk(g[L]),
                       L == 1 ? c->mg_partials : (double*)nullptr, ds);
  return hipGetLastError();
}

// Even-parity PCG iteration with the multigrid preconditioner: w_o | alpha |
// r update (<r, M r>, <r, r> partials) | V-cycle | scalars (stop test, beta) | x, p.
static hipError_t enqueue_iteration_mg(pn_ctx* c, hipStream_t st) {
  StencilArgs a = base_args(c);
  a.st = c->st;
  a.tsign = 1.0;
  a.partials = c->partials;
  a.x = c->p32; a.y = c->p32;
  hipError_t e = launch_stencil<float, M_ODD_W, float>(c, a, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fin_alpha_pcg, dim3(1), dim3(kFinBlock), 0, st, c->st, c->partials, c->nblocks);
  a.x = c->p32; a.y = c->r32[1]; a.m16 = c->m16;
  e = launch_stencil<float, M_EVEN_SR, float>(c, a, st);
  if (e != hipSuccess) return e;
  e = mg_vcycle(c, c->r32[1], st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fin_iter_mg, dim3(1), dim3(kFinBlock), 0, st, c->st, (const double*)c->partials, c->nblocks,
                     (const double*)c->mg_partials, c->mg_npart, (double)kMgOmegaFine);
  const dim3 vg(pcg_vec_blocks(c), c->even.nk);
  hipLaunchKernelGGL(k_pcg_vec_mg<2>, vg, dim3(kBlock), 0, st, c->d32, (const float*)c->r32[1], c->p32,
                     (const uint16_t*)c->m16, c->mg_fine, c->mg_geom[1], mg_final(c, 1), kMgOmegaFine,
                     (const DevState*)c->st);
  return hipGetLastError();
}

static pn_status build_graph_mg(pn_ctx* c, int iters, hipGraphExec_t* exec) {
  hipGraph_t g = nullptr;
  PN_HIP(hipStreamBeginCapture(c->sstream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int i = 0; i < iters && e == hipSuccess; ++i) e = enqueue_iteration_mg(c, c->sstream);
  hipError_t e2 = hipStreamEndCapture(c->sstream, &g);
  if (e != hipSuccess) { if (g) hipGraphDestroy(g); return fail(c, PN_ERR_HIP, std::string("capture: ") + hipGetErrorString(e)); }
  if (e2 != hipSuccess) return fail(c, PN_ERR_HIP, std::string("end capture: ") + hipGetErrorString(e2));
  hipError_t e3 = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e3 != hipSuccess) return fail(c, PN_ERR_HIP, std::string("instantiate: ") + hipGetErrorString(e3));
  return PN_OK;
}

static pn_status build_graph_cg(pn_ctx* c, int iters, bool eq, hipGraphExec_t* exec) {
  hipGraph_t g = nullptr;
  PN_HIP(hipStreamBeginCapture(c->sstream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int i = 0; i < iters && e == hipSuccess; ++i)
    e = enqueue_iteration_cg(c, c->d32, c->p32, c->q32, c->s32, eq, c->sstream);
  hipError_t e2 = hipStreamEndCapture(c->sstream, &g);
  if (e != hipSuccess) { if (g) hipGraphDestroy(g); return fail(c, PN_ERR_HIP, std::string("capture: ") + hipGetErrorString(e)); }
  if (e2 != hipSuccess) return fail(c, PN_ERR_HIP, std::string("end capture: ") + hipGetErrorString(e2));
  hipError_t e3 = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e3 != hipSuccess) return fail(c, PN_ERR_HIP, std::string("instantiate: ") + hipGetErrorString(e3));
  return PN_OK;
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

// ------------------------------------------------------ learned network --
static NetGeom net_geom(const pn_ctx* c, bool padded) {
  NetGeom g;
  std::memset(&g, 0, sizeof(g));
  g.nx = c->nx; g.ny = c->ny; g.nz = c->nz;
  g.nx8 = (c->nx + 7) / 8 * 8; g.ny8 = (c->ny + 7) / 8 * 8; g.nz8 = (c->nz + 7) / 8 * 8;
  g.CX = c->nx + 2; g.CY = c->ny + 2;
  g.nk = std::min(kNetOut, c->nc);
  g.h = c->h;
  for (int k = 0; k < g.nk; ++k) {
    if (padded) {
      g.base[k] = (long long)k * c->cs + ((long long)c->PY + 1) * c->PX + 1;
      g.sy[k] = c->PX;
      g.sz[k] = c->plane;
    } else {
      g.base[k] = c->off[k];
      g.sy[k] = c->ext[k][0];
      g.sz[k] = (long long)c->ext[k][0] * c->ext[k][1];
    }
  }
  return g;
}

static pn_status ensure_small_net_bufs(pn_ctx* c) {
  if (!c->absmax) PN_HIP(hipMalloc(&c->absmax, sizeof(unsigned)));
  if (!c->sq_part) PN_HIP(hipMalloc(&c->sq_part, sizeof(double) * 1024));
  return PN_OK;
}

static pn_status ensure_net_bufs(pn_ctx* c) {
  pn_status e = ensure_small_net_bufs(c);
  if (e != PN_OK) return e;
  if (c->net_x) return PN_OK;
  const NetGeom g = net_geom(c, true);
  const long long v8 = (long long)g.nx8 * g.ny8 * g.nz8;
  PN_HIP(hipMalloc(&c->net_x, sizeof(uint16_t) * v8 * nn::kC));
  PN_HIP(hipMalloc(&c->net_y, sizeof(float) * v8 * nn::kC));
  PN_HIP(hipMalloc(&c->u64, sizeof(double) * c->nv));
  PN_HIP(hipMalloc(&c->w64, sizeof(double) * c->nv));
  PN_HIP(hipMemsetAsync(c->w64, 0, sizeof(double) * c->nv, c->stream));
  PN_HIP(hipMalloc(&c->st_net, sizeof(DevState)));
  PN_HIP(hipMemsetAsync(c->st_net, 0, sizeof(DevState), c->stream));
  PN_HIP(hipStreamSynchronize(c->stream));
  return PN_OK;
}

static int cells_grid(const NetGeom& g) {
  const long long n = (long long)g.nx * g.ny * g.nz * g.nk;
  long long b = (n + kBlock - 1) / kBlock;
  return (int)std::max(1LL, std::min(b, 1024LL));
}

static pn_status launch_features(pn_ctx* c, const float* src, const NetGeom& g, uint16_t* x, hipStream_t s) {
  PN_HIP(hipMemsetAsync(c->absmax, 0, sizeof(unsigned), s));
  hipLaunchKernelGGL(k_src_absmax, dim3(cells_grid(g)), dim3(kBlock), 0, s, src, g, c->absmax);
  const long long v8 = (long long)g.nx8 * g.ny8 * g.nz8;
  hipLaunchKernelGGL(k_net_features, dim3(grid_for(v8)), dim3(kBlock), 0, s, (const float2*)c->med, src, g,
                     (const unsigned*)c->absmax, x);
  PN_HIP(hipGetLastError());
  return PN_OK;
}

// u64 <- the network's prediction for the medium and a padded FP32 source.
static pn_status net_predict(pn_ctx* c, const float* src_pad, hipStream_t s) {
  const NetGeom g = net_geom(c, true);
  pn_status e = launch_features(c, src_pad, g, c->net_x, s);
  if (e != PN_OK) return e;
  void* own = pn_net_get_stream(c->net);
  pn_net_set_stream(c->net, s);
  e = pn_net_forward(c->net, 1, g.nx8, g.ny8, g.nz8, c->net_x, c->net_y);
  pn_net_set_stream(c->net, own);
  if (e != PN_OK) return fail(c, e, std::string("network: ") + pn_net_last_error(c->net));
  hipLaunchKernelGGL((k_fill<double>), dim3(grid_for(c->nv)), dim3(kBlock), 0, s, c->u64, (long)c->nv, 0.0);
  hipLaunchKernelGGL(k_net_to_lattice, dim3(grid_for((long long)g.nx * g.ny * g.nz * g.nk)), dim3(kBlock), 0, s,
                     (const float*)c->net_y, g, c->u64);
  PN_HIP(hipGetLastError());
  return PN_OK;
}

// s minimising ||rhs - s A u64||_2 (rhs padded FP32) and the ratio of the
// residual norms after / before, from ||A u||^2, ||rhs - A u||^2, ||rhs||^2.
// The sums go through st_net: the Krylov scalars in st stay untouched, so a
// rejected step leaves the refinement exactly as it was.
static pn_status net_scale(pn_ctx* c, const float* rhs_pad, hipStream_t s, double* sopt, double* ratio) {
  StencilArgs a = base_args(c);
  a.x = c->u64; a.y = c->w64; a.partials = c->partials;
  PN_HIP((launch_stencil<double, M_APPLY, double>(c, a, s)));
  hipLaunchKernelGGL(k_fin_resid, dim3(1), dim3(kFinBlock), 0, s, c->st_net, c->partials, c->nblocks);
  PN_HIP(hipMemcpyAsync(c->st_host, c->st_net, sizeof(DevState), hipMemcpyDeviceToHost, s));
  PN_HIP(hipStreamSynchronize(s));
  const double au2 = c->st_host->rtrue2;
  a = base_args(c);
  a.x = c->u64; a.x2 = rhs_pad; a.y = c->r32[1]; a.partials = c->partials;
  PN_HIP((launch_stencil<double, M_RESID, float>(c, a, s)));
  hipLaunchKernelGGL(k_fin_resid, dim3(1), dim3(kFinBlock), 0, s, c->st_net, c->partials, c->nblocks);
  PN_HIP(hipMemcpyAsync(c->st_host, c->st_net, sizeof(DevState), hipMemcpyDeviceToHost, s));
  PN_HIP(hipStreamSynchronize(s));
  const double rr = c->st_host->rtrue2, bb = c->st_host->bb2;
  *sopt = 0.0;
  *ratio = 1.0;
  if (au2 > 0.0 && bb > 0.0 && std::isfinite(au2) && std::isfinite(rr)) {
    const double dot = 0.5 * (bb + au2 - rr);
    *sopt = dot / au2;
    *ratio = std::sqrt(std::max(0.0, bb - dot * dot / au2) / bb);
  }
  return PN_OK;
}

extern "C" pn_status pn_attach_net(pn_ctx* c, pn_net* net) {
  if (!c) return PN_ERR_ARG;
  if (!c->p32) return fail(c, PN_ERR_ARG, "context has no Krylov workspace (a batch problem context)");
  c->net = net;
  return PN_OK;
}

extern "C" pn_status pn_net_grid(const pn_ctx* c, int* nx8, int* ny8, int* nz8) {
  if (!c || !nx8 || !ny8 || !nz8) return PN_ERR_ARG;
  *nx8 = (c->nx + 7) / 8 * 8;
  *ny8 = (c->ny + 7) / 8 * 8;
  *nz8 = (c->nz + 7) / 8 * 8;
  return PN_OK;
}

extern "C" pn_status pn_net_features(pn_ctx* c, const float* src, uint16_t* x) {
  if (!c) return PN_ERR_ARG;
  if (!src || !x) return fail(c, PN_ERR_ARG, "src or x is NULL");
  pn_status e = ensure_small_net_bufs(c);
  if (e != PN_OK) return e;
  return launch_features(c, src, net_geom(c, false), x, c->stream);
}

extern "C" pn_status pn_net_targets_diff(pn_ctx* c, const double* sol, const double* sub, uint16_t* t) {
  if (!c) return PN_ERR_ARG;
  if (!sol || !t) return fail(c, PN_ERR_ARG, "solution or t is NULL");
  pn_status e = ensure_small_net_bufs(c);
  if (e != PN_OK) return e;
  const NetGeom g = net_geom(c, false);
  const int nb = cells_grid(g);
  hipLaunchKernelGGL(k_coef0_absmax, dim3(nb), dim3(kBlock), 0, c->stream, sol, sub, g, c->sq_part);
  const long long n = (long long)g.nx8 * g.ny8 * g.nz8 * kNetOut;
  hipLaunchKernelGGL(k_net_targets, dim3(grid_for(n)), dim3(kBlock), 0, c->stream, sol, sub, g,
                     (const double*)c->sq_part, nb, t);
  PN_HIP(hipGetLastError());
  return PN_OK;
}

extern "C" pn_status pn_net_targets(pn_ctx* c, const double* sol, uint16_t* t) {
  return pn_net_targets_diff(c, sol, nullptr, t);
}

template <typename T>
static const float* r0_as_float(const T* r) {
  if constexpr (sizeof(T) == 4) return r;
  else return nullptr;  // learned steps run in the FP32 solve only
}

static double ms_since(const std::chrono::steady_clock::time_point& t) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
}

// Iterative refinement around CGLS on the padded lattice.  b32 holds Q and
// x64 the FP64 iterate on entry; x64 holds the result on exit.
template <typename T>
static pn_status solve_impl(pn_ctx* c, double tol, const pn_solve_opts& o, pn_solve_info* info) {
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
  // FP32, variant CG: CG on the normal equations with the recursive normal
  // residual (10 vector passes per iteration, the A^T pass streams one
  // vector); otherwise CGLS with the recursive residual r (11 passes, r
  // ping-pong, the A^T pass streams two).
  // FP32 even-parity PCG (Schur complement): SCHUR, and AUTO on the
  // register-window stencil when no axis is Neumann
  // with the multigrid preconditioner: SCHUR_MG, and AUTO for large odd-order problems
  const bool mg = (sizeof(T) == 4) && mg_ok(c) && !c->use_lds &&
                  (o.variant == PN_VARIANT_SCHUR_MG || (o.variant == PN_VARIANT_AUTO && mg_auto(c)));
  const bool schur = (sizeof(T) == 4) && schur_ok(c) &&
                     (mg || o.variant == PN_VARIANT_SCHUR || (o.variant == PN_VARIANT_AUTO && !c->use_lds));
  const bool cg = (sizeof(T) == 4) && !schur && o.variant != PN_VARIANT_CGLS;
  // row equilibration: AUTO and CG_EQ on the register-window stencil
  const bool eq = cg && !c->use_lds && (o.variant == PN_VARIANT_AUTO || o.variant == PN_VARIANT_CG_EQ);
  if (cg) {
    gexec = &c->gexec_cg;
    giters = &c->giters_cg;
  }
  if (schur) {
    gexec = mg ? &c->gexec_mg : &c->gexec_schur;
    giters = mg ? &c->giters_mg : &c->giters_schur;
  }
  if (mg) {
    pn_status e = mg_alloc(c);
    if (e != PN_OK) return e;
  }
  int gi = o.graph_iters < 2 ? 2 : (o.graph_iters + 1) & ~1;  // even: r ends in r0
  if (*gexec == nullptr || *giters != gi || (cg && c->gcg_eq != (int)eq)) {
    if (*gexec) { hipGraphExecDestroy(*gexec); *gexec = nullptr; }
    pn_status e = mg      ? build_graph_mg(c, gi, gexec)
                  : schur ? build_graph_schur(c, gi, gexec)
                  : cg  ? build_graph_cg(c, gi, eq, gexec)
                        : build_graph<T>(c, gi, d, p, q, s, r0, r1, gexec);
    if (e != PN_OK) return e;
    *giters = gi;
    if (cg) c->gcg_eq = (int)eq;
  }
  const dim3 vg(pcg_vec_blocks(c), c->even.nk);
  if (schur) {
    pn_status e = schur_prepare(c, mg, c->sstream);
    if (e != PN_OK) return e;
  }
  hipStream_t ss = c->sstream;
  DevState init;
  std::memset(&init, 0, sizeof(init));
  init.max_iters = o.max_iter;
  PN_HIP(hipMemcpyAsync(c->st, &init, sizeof(DevState), hipMemcpyHostToDevice, ss));
  PN_HIP(hipStreamSynchronize(ss));
  pn_status result = PN_ERR_NOT_CONVERGED;
  int outer = 0;
  double rel = 0.0, bnorm = 0.0;
  if (info) info->nhistory = 0;
  // learned start: x = s u with u the network's prediction for (medium, Q)
  const bool learned = sizeof(T) == 4 && c->net != nullptr && o.learned != PN_LEARNED_OFF;
  if (learned) {
    pn_status e = ensure_net_bufs(c);
    if (e != PN_OK) return e;
  }
  double t_res = 0.0, t_kry = 0.0, t_net = 0.0;
  int starts = 0;
  if (learned && !o.use_guess) {
    const auto tl = std::chrono::steady_clock::now();
    double sc = 0.0, ratio = 1.0;
    pn_status e = net_predict(c, c->b32, ss);
    if (e == PN_OK) e = net_scale(c, c->b32, ss, &sc, &ratio);
    if (e != PN_OK) return e;
    if (info) info->learned_ratio = ratio;
    if (ratio < 0.9 && std::isfinite(sc)) {  // a weak guess only changes the error's make-up
      hipLaunchKernelGGL(k_axpby64, dim3(grid_for(c->nv)), dim3(kBlock), 0, ss, c->x64, (const double*)c->u64, 0.0,
                         sc, (long)c->nv);
      PN_HIP(hipGetLastError());
      if (info) info->learned_steps += 1;
    }
    t_net += ms_since(tl);
  }
  bool corrected = false;
  for (;;) {
    const auto tr = std::chrono::steady_clock::now();
    pn_status e = residual<T>(c, c->b32, c->x64, r0, ss);
    if (e != PN_OK) return e;
    PN_HIP(hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, ss));
    PN_HIP(hipStreamSynchronize(ss));
    t_res += ms_since(tr);
    const DevState h = *c->st_host;
    ++outer;
    bnorm = std::sqrt(h.bb2);
    if (h.bb2 == 0.0) {  // Q = 0: the solution is 0
      hipLaunchKernelGGL((k_fill<double>), dim3(grid_for(c->nv)), dim3(kBlock), 0, ss, c->x64, (long)c->nv, 0.0);
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
    // learned correction x += s u, u the prediction for the residual r0
    if (learned && o.learned == PN_LEARNED_GUESS_CORRECT && !corrected) {
      const auto tl = std::chrono::steady_clock::now();
      double sc = 0.0, ratio = 1.0;
      pn_status e = net_predict(c, r0_as_float(r0), ss);
      if (e == PN_OK) e = net_scale(c, r0_as_float(r0), ss, &sc, &ratio);
      if (e != PN_OK) return e;
      t_net += ms_since(tl);
      if (ratio < 0.9 && std::isfinite(sc)) {
        hipLaunchKernelGGL(k_axpby64, dim3(grid_for(c->nv)), dim3(kBlock), 0, ss, c->x64, (const double*)c->u64, 1.0,
                           sc, (long)c->nv);
        PN_HIP(hipGetLastError());
        if (info) info->learned_steps += 1;
        corrected = true;
        continue;  // re-evaluate the FP64 residual
      }
    }
    corrected = false;
    const auto tk = std::chrono::steady_clock::now();
    ++starts;
    // inner solve  A d = r0  from d = 0
    // relative reduction asked of this inner solve: inner_tol, but no further
    // than the outer tolerance needs (FP64 Krylov: all the way)
    double itol = std::max(o.inner_tol, 0.3 * tol / rel);
    if constexpr (sizeof(T) == 8) itol = 0.5 * tol / rel;
    if (itol >= 1.0) itol = 0.5;
    hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(c->nv)), dim3(kBlock), 0, ss, d, (long)c->nv, T(0));
    StencilArgs a = base_args(c);
    a.partials = c->partials;
    if constexpr (sizeof(T) == 4) {
      if (schur) {
        // reduced right-hand side f = r0_e - T_eo D_o^-1 r0_o (u_o = D_o^-1 r0_o
        // in the odd slots of q32, f in the even slots of r32[1])
        StencilArgs b = base_args(c);
        b.x = d; b.x2 = r0; b.y = q;
        PN_HIP((launch_stencil<float, M_ODD_BACK, float>(c, b, ss)));
        b.x = q; b.x2 = r0; b.y = r1;
        PN_HIP((launch_stencil<float, M_EVEN_RHS, float>(c, b, ss)));
        hipLaunchKernelGGL(k_pcg_vec<0>, vg, dim3(kBlock), 0, ss, d, r1, p, (const float*)q, (const uint16_t*)c->m16,
                           c->even, c->partials, (const DevState*)c->st);
        if (mg) {  // p = B r, gamma = <r, B r>
          hipLaunchKernelGGL(k_fin_rz_mg<true>, dim3(1), dim3(kFinBlock), 0, ss, c->st, (const double*)c->partials,
                             (int)(vg.x * vg.y), itol * itol);
          PN_HIP(mg_vcycle(c, r1, ss));
          hipLaunchKernelGGL(k_fin_beta_mg<true>, dim3(1), dim3(kFinBlock), 0, ss, c->st,
                             (const double*)c->mg_partials, c->mg_npart, (double)kMgOmegaFine);
          hipLaunchKernelGGL(k_pcg_vec_mg<4>, vg, dim3(kBlock), 0, ss, d, (const float*)r1, p,
                             (const uint16_t*)c->m16, c->mg_fine, c->mg_geom[1], mg_final(c, 1), kMgOmegaFine,
                             (const DevState*)c->st);
        } else {
          hipLaunchKernelGGL(k_fin_init_pcg, dim3(1), dim3(kFinBlock), 0, ss, c->st, c->partials, (int)(vg.x * vg.y),
                             itol * itol);
        }
        PN_HIP(hipGetLastError());
        for (;;) {
          PN_HIP(hipGraphLaunch(*gexec, ss));
          PN_HIP(hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, ss));
          PN_HIP(hipStreamSynchronize(ss));
          if (c->st_host->done || c->st_host->stop) break;
        }
        // odd part: d_o = (r0_o - T_oe d_e) / d_o
        b.x = d; b.x2 = r0; b.y = d;
        PN_HIP((launch_stencil<float, M_ODD_BACK, float>(c, b, ss)));
        hipLaunchKernelGGL((k_axpy64<T>), dim3(grid_for(c->nv)), dim3(kBlock), 0, ss, c->x64, (const T*)d, (long)c->nv);
        PN_HIP(hipGetLastError());
        t_kry += ms_since(tk);
        continue;
      }
    }
    const T* rs = r0;
    if constexpr (sizeof(T) == 4) {
      if (eq) {  // r1 = W r0; the inner solve tracks <r, W r>
        a.x = r0; a.y = r1;
        PN_HIP((launch_stencil<float, M_EQS, float>(c, a, ss)));
        hipLaunchKernelGGL(k_fin_rr, dim3(1), dim3(kFinBlock), 0, ss, c->st, c->partials, c->nblocks);
        PN_HIP(hipGetLastError());
        rs = r1;
      }
    }
    a.x = rs; a.y = s; a.tsign = -1.0;
    if (cg && c->use_lds) PN_HIP(launch_lds(c, M_APPLY, true, a, ss));
    else PN_HIP((launch_stencil<T, M_APPLY, T>(c, a, ss)));
    hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(kFinBlock), 0, ss, c->st, c->partials,
                       (cg && c->use_lds) ? c->lnblocks : c->nblocks, itol * itol);
    PN_HIP(hipGetLastError());
    PN_HIP(hipMemcpyAsync(p, s, sizeof(T) * c->nv, hipMemcpyDeviceToDevice, ss));  // p = s
    for (;;) {
      PN_HIP(hipGraphLaunch(*gexec, ss));
      PN_HIP(hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, ss));
      PN_HIP(hipStreamSynchronize(ss));
      if (c->st_host->done || c->st_host->stop) break;
    }
    hipLaunchKernelGGL((k_axpy64<T>), dim3(grid_for(c->nv)), dim3(kBlock), 0, ss, c->x64, (const T*)d, (long)c->nv);
    PN_HIP(hipGetLastError());
    t_kry += ms_since(tk);
  }
  if (info) {
    info->status = result;
    info->outer_iters = outer;
    info->inner_iters = c->st_host->iters;
    info->rel_residual = rel;
    info->bnorm = bnorm;
    info->t_ms[PN_PHASE_RESIDUAL] = t_res;
    info->t_ms[PN_PHASE_KRYLOV] = t_kry;
    info->t_ms[PN_PHASE_LEARNED] = t_net;
    const SolveBytes sb = schur ? schur_bytes(c, mg) : solve_bytes(c, sizeof(T) == 8, cg, eq);
    info->bytes = sb.per_iter * info->inner_iters + sb.per_start * starts + sb.per_resid * outer;
    info->achieved_gbs = (t_res + t_kry) > 0.0 ? info->bytes / ((t_res + t_kry) * 1e6) : 0.0;
  }
  return result;
}

pn_status solve_padded_mg(pn_ctx* c, double tol, const pn_solve_opts& o, pn_solve_info* info) {
  if (o.variant != PN_VARIANT_SCHUR_MG || o.precision != PN_FP32_IR || !mg_ok(c) || c->use_lds)
    return fail(c, PN_ERR_ARG, "the padded multigrid solve needs PN_VARIANT_SCHUR_MG, FP32_IR and no Neumann axis");
  if (info) std::memset(info, 0, sizeof(*info));
  const auto t0 = std::chrono::steady_clock::now();
  pn_status s = solve_impl<float>(c, tol, o, info);
  PN_HIP(hipStreamSynchronize(c->sstream));
  if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return s;
}

bool mg_supported(const pn_ctx* c) { return c && mg_ok(c) && !c->use_lds; }

pn_status prepare_mg_solve(pn_ctx* c, const pn_solve_opts& o) {
  pn_status e = mg_alloc(c);
  if (e != PN_OK) return e;
  const int gi = o.graph_iters < 2 ? 2 : (o.graph_iters + 1) & ~1;  // as solve_impl
  if (c->gexec_mg == nullptr || c->giters_mg != gi) {
    if (c->gexec_mg) { hipGraphExecDestroy(c->gexec_mg); c->gexec_mg = nullptr; }
    e = build_graph_mg(c, gi, &c->gexec_mg);
    if (e != PN_OK) return e;
    c->giters_mg = gi;
  }
  PN_HIP(hipStreamSynchronize(c->sstream));
  return PN_OK;
}

pn_status borrow_workspace(pn_ctx* c, void* const* v) {
  float** dst[6] = {&c->r32[0], &c->r32[1], &c->s32, &c->p32, &c->q32, &c->d32};
  for (int i = 0; i < 6; ++i) *dst[i] = static_cast<float*>(v[i]);
  if (!c->m16) {
    PN_HIP(hipMalloc(&c->m16, sizeof(uint16_t) * c->nv));
    PN_HIP(hipMemsetAsync(c->m16, 0, sizeof(uint16_t) * c->nv, c->sstream));
  }
  if (!c->st) PN_HIP(hipMalloc(&c->st, sizeof(DevState)));
  if (!c->st_host) PN_HIP(hipHostMalloc(&c->st_host, sizeof(DevState), hipHostMallocDefault));
  if (!c->partials) PN_HIP(hipMalloc(&c->partials, sizeof(double) * 2 * c->max_blocks));
  PN_HIP(hipStreamSynchronize(c->sstream));
  return PN_OK;
}

void unborrow_workspace(pn_ctx* c) {
  c->r32[0] = c->r32[1] = c->s32 = c->p32 = c->q32 = c->d32 = c->b32 = nullptr;
  c->x64 = nullptr;
}

extern "C" pn_status pn_solve(pn_ctx* c, const float* rhs, double* x, double tol, const pn_solve_opts* opts,
                              pn_solve_info* info) {
  if (!c) return PN_ERR_ARG;
  if (!c->p32) return fail(c, PN_ERR_ARG, "context has no Krylov workspace (a batch problem context)");
  if (!rhs || !x) return fail(c, PN_ERR_ARG, "rhs or x is NULL");
  if (!(tol > 0.0)) return fail(c, PN_ERR_ARG, "tol must be > 0");
  pn_solve_opts o;
  pn_default_opts(&o);
  if (opts) o = *opts;
  if (o.max_iter < 1 || o.max_refine < 0 || !(o.inner_tol > 0.0 && o.inner_tol < 1.0))
    return fail(c, PN_ERR_ARG, "invalid solve options");
  if (o.precision != PN_FP32_IR && o.precision != PN_FP64) return fail(c, PN_ERR_ARG, "unknown precision");
  if (o.learned < PN_LEARNED_OFF || o.learned > PN_LEARNED_GUESS_CORRECT)
    return fail(c, PN_ERR_ARG, "unknown learned mode");
  if (o.variant < PN_VARIANT_AUTO || o.variant > PN_VARIANT_SCHUR_MG) return fail(c, PN_ERR_ARG, "unknown variant");
  if (o.variant == PN_VARIANT_SCHUR && (!schur_ok(c) || o.precision != PN_FP32_IR))
    return fail(c, PN_ERR_ARG, "the even-parity Schur variant needs FP32_IR, no Neumann axis and positive extinction");
  if (o.variant == PN_VARIANT_SCHUR_MG && (!mg_ok(c) || c->use_lds || o.precision != PN_FP32_IR))
    return fail(c, PN_ERR_ARG, "the multigrid even-parity variant needs FP32_IR, the register-window stencil, no "
                               "Neumann axis and positive extinction");
  if (o.variant == PN_VARIANT_CG_EQ && (c->use_lds || o.precision != PN_FP32_IR))
    return fail(c, PN_ERR_ARG, "the equilibrated CG variant needs FP32_IR and the register-window stencil");
  if (info) std::memset(info, 0, sizeof(*info));
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t ss = c->sstream;
  // order the solve after the caller's pending work
  PN_HIP(hipEventRecord(c->ev_in, c->stream));
  PN_HIP(hipStreamWaitEvent(ss, c->ev_in, 0));
  // non-finite right-hand side
  PN_HIP(hipMemsetAsync(c->flag, 0, sizeof(int), ss));
  hipLaunchKernelGGL(k_check_finite, dim3(grid_for(c->n)), dim3(kBlock), 0, ss, rhs, c->n, c->flag);
  PN_HIP(hipGetLastError());
  PN_HIP(hipMemcpyAsync(c->flag_host, c->flag, sizeof(int), hipMemcpyDeviceToHost, ss));
  PN_HIP(hipStreamSynchronize(ss));
  if (*c->flag_host) return fail(c, PN_ERR_NONFINITE, "right-hand side contains NaN or Inf");
  // packed -> padded: Q into b32, the initial iterate into x64
  PN_HIP((launch_pack<float, float, 0>(c, rhs, c->b32, ss)));
  if (o.use_guess) {
    PN_HIP((launch_pack<double, double, 0>(c, x, c->x64, ss)));
  } else {
    hipLaunchKernelGGL((k_fill<double>), dim3(grid_for(c->nv)), dim3(kBlock), 0, ss, c->x64, (long)c->nv, 0.0);
    PN_HIP(hipGetLastError());
  }
  PN_HIP(hipStreamSynchronize(ss));
  const double t_setup = ms_since(t0);
  pn_status s = (o.precision == PN_FP64) ? solve_impl<double>(c, tol, o, info) : solve_impl<float>(c, tol, o, info);
  const auto tf = std::chrono::steady_clock::now();
  // padded -> packed result (also after a failed solve: x is the last iterate)
  PN_HIP((launch_pack<double, double, 1>(c, c->x64, x, ss)));
  PN_HIP(hipEventRecord(c->ev_out, ss));
  PN_HIP(hipStreamWaitEvent(c->stream, c->ev_out, 0));
  PN_HIP(hipStreamSynchronize(ss));
  if (info) {
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->t_ms[PN_PHASE_SETUP] = t_setup;
    info->t_ms[PN_PHASE_FINISH] = ms_since(tf);
  }
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
