// Batched solve: many media of uneven grid size and order, each with several
// right-hand sides, advanced together by one captured graph of Krylov
// iterations (declarations in include/pn.h).
//
// A system is one (problem, right-hand side) pair.  Every stage of the
// mixed-precision CGLS iteration is ONE launch over all systems of an order
// (stencil) or over all systems (scalars, vector updates): the kernels take a
// work list of (system, tile) items and a device table of per-system
// arguments, and every system keeps its own device scalars, so systems
// converge, stop and are skipped independently.  The arithmetic per system is
// exactly that of pn_solve with the same launch geometry.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <thread>
#include <vector>

#include "pn_internal.h"

namespace {

// Host threads of the batched multigrid path (at most the host's hardware
// threads): more than the GPU's hardware queues, since each thread waits on
// the host for its problem's stop flag after every captured graph (48 x 8
// systems: 4 threads 3.81 s, 8 threads 3.71 s, 16 threads 3.62 s).
constexpr int kMgThreads = 16;

struct Group {
  int order = 0, gen = 0;  // gen: some axis is not vacuum (general-boundary kernels)
  int2* work = nullptr;         // device list of the systems in the current launch set
  int nwork = 0;
  std::vector<int2> full;       // every (system, tile) of the group
};

}  // namespace

struct pn_batch {
  int nprob = 0, nrhs = 0, nsys = 0;
  hipStream_t stream = nullptr;   // caller's stream
  hipStream_t sstream = nullptr;  // solve stream (capture)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<pn_ctx*> prob;      // geometry and medium per problem
  std::vector<void*> arena;       // vectors of one system
  std::vector<SysArgs> sys_h;
  SysArgs* sys = nullptr;
  DevState* st = nullptr;
  DevState* st_host = nullptr;
  double* partials = nullptr;
  int* active = nullptr;
  int* active_host = nullptr;
  int* flag = nullptr;
  int* flag_host = nullptr;
  std::vector<Group> groups;
  int2* vwork = nullptr;
  int nvwork = 0;
  std::vector<int2> vfull;        // every (system, chunk)
  int nlaunch = 0;                // systems in the current launch set
  hipGraphExec_t gexec = nullptr;
  int giters = 0;
  bool gcg = false;
  bool geq = false;
  long long unknowns = 0;
  std::string err;
};

namespace {

thread_local std::string g_batch_error;

pn_status bfail(pn_batch* b, pn_status s, const std::string& m) {
  if (b) b->err = m; else g_batch_error = m;
  return s;
}

#define B_HIP(call)                                                                     \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return bfail(b, e_ == hipErrorOutOfMemory ? PN_ERR_ALLOC : PN_ERR_HIP,            \
                   std::string(#call) + ": " + hipGetErrorString(e_));                  \
  } while (0)

void free_batch(pn_batch* b) {
  if (!b) return;
  if (b->gexec) hipGraphExecDestroy(b->gexec);
  for (void* p : b->arena) hipFree(p);
  for (pn_ctx* c : b->prob) free_ctx(c);
  for (Group& g : b->groups) hipFree(g.work);
  hipFree(b->vwork);
  hipFree(b->sys);
  hipFree(b->st);
  hipFree(b->partials);
  hipFree(b->active);
  hipFree(b->flag);
  if (b->st_host) hipHostFree(b->st_host);
  if (b->active_host) hipHostFree(b->active_host);
  if (b->flag_host) hipHostFree(b->flag_host);
  if (b->ev_in) hipEventDestroy(b->ev_in);
  if (b->ev_out) hipEventDestroy(b->ev_out);
  if (b->sstream) hipStreamDestroy(b->sstream);
  delete b;
}

hipError_t launch_group(const Group& g, int kind, const BatchLaunch& proto, hipStream_t s) {
  BatchLaunch bl = proto;
  bl.work = g.work;
  bl.nwork = g.nwork;
  const bool gen = g.gen != 0;
  switch (g.order) {
    case 1: return launch_batch_order<1>(kind, gen, bl, s);
    case 2: return launch_batch_order<2>(kind, gen, bl, s);
    case 3: return launch_batch_order<3>(kind, gen, bl, s);
    case 4: return launch_batch_order<4>(kind, gen, bl, s);
    case 5: return launch_batch_order<5>(kind, gen, bl, s);
    case 6: return launch_batch_order<6>(kind, gen, bl, s);
    case 7: return launch_batch_order<7>(kind, gen, bl, s);
    default: return hipErrorInvalidValue;
  }
}

BatchLaunch roles(const pn_batch* b, int ix, int ix2, int iy, int iy2, double tsign, int gate) {
  BatchLaunch bl;
  std::memset(&bl, 0, sizeof(bl));
  bl.sys = b->sys;
  bl.ix = ix; bl.ix2 = ix2; bl.iy = iy; bl.iy2 = iy2;
  bl.tsign = tsign;
  bl.gate = gate;
  return bl;
}

hipError_t stencil_all(const pn_batch* b, int kind, const BatchLaunch& bl, hipStream_t s) {
  for (const Group& g : b->groups) {
    if (g.nwork == 0) continue;
    hipError_t e = launch_group(g, kind, bl, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int OP>
hipError_t vec_all(const pn_batch* b, hipStream_t s) {
  if (b->nvwork == 0) return hipSuccess;
  hipLaunchKernelGGL((k_vec_batch<OP>), dim3(b->nvwork), dim3(kBlock), 0, s, (const SysArgs*)b->sys,
                     (const int2*)b->vwork, b->nvwork);
  return hipGetLastError();
}

template <int WHICH>
hipError_t fin_all(const pn_batch* b, hipStream_t s) {
  hipLaunchKernelGGL((k_fin_batch<WHICH>), dim3(b->nsys), dim3(kFinBlock), 0, s, (const SysArgs*)b->sys);
  return hipGetLastError();
}

// One Krylov iteration of every running system, as pn_solve's FP32 inner
// solve: CG on the normal equations (s -= alpha A^T q; eq: row-equilibrated,
// q = W A p), or CGLS (r ping-pong rin -> rout, r' = r - alpha q fused into
// s = A^T r').
hipError_t enqueue_batch_iteration(const pn_batch* b, bool cg, bool eq, int rin, int rout, hipStream_t s) {
  hipError_t e = stencil_all(b, (cg && eq) ? K_F32_APPLY_EQ : K_F32_APPLY, roles(b, BV_P, -1, BV_Q, -1, 1.0, 1), s);
  if (cg) {
    if (e == hipSuccess) e = fin_all<BF_ALPHA_CG>(b, s);
    if (e == hipSuccess) e = stencil_all(b, K_F32_SUPD, roles(b, BV_Q, -1, BV_S, -1, -1.0, 1), s);
    if (e == hipSuccess) e = fin_all<BF_BETA_CG>(b, s);
  } else {
    if (e == hipSuccess) e = fin_all<BF_ALPHA>(b, s);
    if (e == hipSuccess) e = stencil_all(b, K_F32_TRANSR, roles(b, rin, BV_Q, BV_S, rout, -1.0, 1), s);
    if (e == hipSuccess) e = fin_all<BF_BETA>(b, s);
  }
  if (e == hipSuccess) e = vec_all<BO_UPDATE_XP>(b, s);
  return e;
}

// Restricts every launch to the systems with keep[i] != 0 (a subset of the
// full work lists, same order) and drops the captured graph.  Blocks of
// finished systems would otherwise still be dispatched, only to return.
pn_status compact(pn_batch* b, const std::vector<char>& keep, hipStream_t s) {
  int n = 0;
  for (char k : keep) n += k ? 1 : 0;
  if (n == b->nlaunch) return PN_OK;
  std::vector<int2> tmp;
  for (Group& g : b->groups) {
    tmp.clear();
    for (const int2& w : g.full)
      if (keep[w.x]) tmp.push_back(w);
    g.nwork = (int)tmp.size();
    if (g.nwork) B_HIP(hipMemcpyAsync(g.work, tmp.data(), sizeof(int2) * tmp.size(), hipMemcpyHostToDevice, s));
    B_HIP(hipStreamSynchronize(s));  // tmp is reused
  }
  tmp.clear();
  for (const int2& w : b->vfull)
    if (keep[w.x]) tmp.push_back(w);
  b->nvwork = (int)tmp.size();
  if (b->nvwork) B_HIP(hipMemcpyAsync(b->vwork, tmp.data(), sizeof(int2) * tmp.size(), hipMemcpyHostToDevice, s));
  B_HIP(hipStreamSynchronize(s));
  b->nlaunch = n;
  if (b->gexec) { hipGraphExecDestroy(b->gexec); b->gexec = nullptr; b->giters = 0; }
  return PN_OK;
}

pn_status build_batch_graph(pn_batch* b, int iters, bool cg, bool eq) {
  if (b->gexec && b->giters == iters && b->gcg == cg && b->geq == eq) return PN_OK;
  if (b->gexec) { hipGraphExecDestroy(b->gexec); b->gexec = nullptr; b->giters = 0; }
  hipGraph_t g = nullptr;
  B_HIP(hipStreamBeginCapture(b->sstream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int i = 0; i < iters && e == hipSuccess; ++i)
    e = (i & 1) ? enqueue_batch_iteration(b, cg, eq, BV_R1, BV_R0, b->sstream)
                : enqueue_batch_iteration(b, cg, eq, BV_R0, BV_R1, b->sstream);
  hipError_t e2 = hipStreamEndCapture(b->sstream, &g);
  if (e != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return bfail(b, PN_ERR_HIP, std::string("capture: ") + hipGetErrorString(e));
  }
  if (e2 != hipSuccess) return bfail(b, PN_ERR_HIP, std::string("end capture: ") + hipGetErrorString(e2));
  hipError_t e3 = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e3 != hipSuccess) return bfail(b, PN_ERR_HIP, std::string("instantiate: ") + hipGetErrorString(e3));
  b->giters = iters;
  b->gcg = cg;
  b->geq = eq;
  return PN_OK;
}

}  // namespace

extern "C" const char* pn_batch_last_error(const pn_batch* b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

extern "C" void pn_batch_destroy(pn_batch* b) {
  if (!b) return;
  if (b->sstream) hipStreamSynchronize(b->sstream);
  if (b->stream) hipStreamSynchronize(b->stream);
  free_batch(b);
}

extern "C" pn_status pn_batch_setup(int nprob, const pn_problem* probs, int nrhs, int tune, void* stream,
                                    pn_batch** out) {
  if (!out) return bfail(nullptr, PN_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (nprob < 1 || !probs) return bfail(nullptr, PN_ERR_ARG, "need at least one problem");
  if (nrhs < 1) return bfail(nullptr, PN_ERR_ARG, "nrhs must be >= 1");
  if ((long long)nprob * nrhs > (1 << 20)) return bfail(nullptr, PN_ERR_ARG, "too many systems");
  pn_batch* b = new pn_batch();
  b->nprob = nprob;
  b->nrhs = nrhs;
  b->nsys = nprob * nrhs;
  b->stream = (hipStream_t)stream;
  auto bail = [&](pn_status s) {
    const std::string m = b->err;
    free_batch(b);
    return bfail(nullptr, s, m);
  };
#define SETUP_B(call)                                                                             \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess) {                                                                       \
      b->err = std::string(#call) + ": " + hipGetErrorString(e_);                                 \
      return bail(e_ == hipErrorOutOfMemory ? PN_ERR_ALLOC : PN_ERR_HIP);                         \
    }                                                                                             \
  } while (0)
  SETUP_B(hipStreamCreateWithFlags(&b->sstream, hipStreamNonBlocking));
  SETUP_B(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
  SETUP_B(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));

  // problems: geometry and medium (no single-system workspace)
  for (int p = 0; p < nprob; ++p) {
    pn_ctx* c = nullptr;
    pn_status s = setup_ctx(probs[p].order, &probs[p].grid, &probs[p].medium, stream, false, &c);
    if (s != PN_OK) {
      b->err = "problem " + std::to_string(p) + ": " + g_setup_error;
      return bail(s);
    }
    b->prob.push_back(c);
  }
  // vectors of every system: 7 FP32 (r0, r1, s, p, q, d, Q) and the FP64 iterate
  for (int p = 0; p < nprob; ++p) {
    const long long nv = b->prob[p]->nv;
    for (int r = 0; r < nrhs; ++r) {
      void* mem = nullptr;
      const size_t bytes = (size_t)nv * (7 * sizeof(float) + sizeof(double));
      SETUP_B(hipMalloc(&mem, bytes));
      b->arena.push_back(mem);
      SETUP_B(hipMemsetAsync(mem, 0, bytes, b->stream));  // zero halo invariant
    }
  }
  auto vec_of = [&](int sidx, int role) -> void* {
    const long long nv = b->prob[sidx / nrhs]->nv;
    char* base = static_cast<char*>(b->arena[sidx]);
    if (role == BV_X64) return base + (size_t)nv * 7 * sizeof(float);
    return base + (size_t)nv * role * sizeof(float);
  };
  // launch geometry: the tune cache, filled first by the autotuner if asked
  if (tune) {
    for (int p = 0; p < nprob; ++p) {
      pn_ctx* c = b->prob[p];
      if (tune_lookup(c, nullptr, nullptr)) continue;
      double ms = 0.0;
      const int z = tune_zchunk(c, (const float*)vec_of(p * nrhs, BV_P), (float*)vec_of(p * nrhs, BV_Q), 10, &ms);
      if (z < 0) { b->err = "autotune: a timing launch failed"; return bail(PN_ERR_HIP); }
      tune_store(c, z, ms);
    }
  }
  for (pn_ctx* c : b->prob) {
    int z = 0;
    set_geometry(c, tune_lookup(c, &z, nullptr) ? z : 0);
    if (c->nblocks > c->max_blocks) set_geometry(c, 0);
  }
  // per-system arguments, scalars and partial sums
  long long npart = 0;
  for (int p = 0; p < nprob; ++p) npart += (long long)b->prob[p]->nblocks * nrhs;
  SETUP_B(hipMalloc(&b->partials, sizeof(double) * 2 * npart));
  SETUP_B(hipMalloc(&b->st, sizeof(DevState) * b->nsys));
  SETUP_B(hipMemsetAsync(b->st, 0, sizeof(DevState) * b->nsys, b->stream));
  SETUP_B(hipHostMalloc(&b->st_host, sizeof(DevState) * b->nsys, hipHostMallocDefault));
  b->sys_h.resize(b->nsys);
  long long poff = 0;
  for (int p = 0; p < nprob; ++p) {
    pn_ctx* c = b->prob[p];
    for (int r = 0; r < nrhs; ++r) {
      const int sidx = p * nrhs + r;
      SysArgs& a = b->sys_h[sidx];
      std::memset(&a, 0, sizeof(a));
      a.a = base_args(c);
      a.a.st = b->st + sidx;
      a.a.partials = b->partials + 2 * poff;
      poff += c->nblocks;
      for (int v = 0; v < BV_COUNT; ++v) a.vec[v] = vec_of(sidx, v);
      a.nv = c->nv;
      b->unknowns += c->n;
    }
  }
  SETUP_B(hipMalloc(&b->sys, sizeof(SysArgs) * b->nsys));
  SETUP_B(hipMemcpyAsync(b->sys, b->sys_h.data(), sizeof(SysArgs) * b->nsys, hipMemcpyHostToDevice, b->stream));
  // stencil work lists, one per (order, boundary): problem, then tile, then rhs
  std::map<std::pair<int, int>, std::vector<int2>> lists;
  for (int p = 0; p < nprob; ++p) {
    pn_ctx* c = b->prob[p];
    auto& w = lists[{c->order, (c->bcs[0] != BC_VACUUM || c->bcs[1] != BC_VACUUM || c->bcs[2] != BC_VACUUM) ? 1 : 0}];
    for (int L = 0; L < c->nblocks; ++L)
      for (int r = 0; r < nrhs; ++r) w.push_back(make_int2(p * nrhs + r, L));
  }
  for (auto& kv : lists) {
    if (kv.second.size() >= (size_t)INT32_MAX) { b->err = "work list too long"; return bail(PN_ERR_ARG); }
    Group g;
    g.order = kv.first.first;
    g.gen = kv.first.second;
    g.nwork = (int)kv.second.size();
    SETUP_B(hipMalloc(&g.work, sizeof(int2) * g.nwork));
    SETUP_B(hipMemcpy(g.work, kv.second.data(), sizeof(int2) * g.nwork, hipMemcpyHostToDevice));
    g.full = std::move(kv.second);
    b->groups.push_back(std::move(g));
  }
  // vector work list: (system, chunk)
  {
    std::vector<int2> vw;
    for (int sidx = 0; sidx < b->nsys; ++sidx) {
      const long long nch = (b->sys_h[sidx].nv + kChunk - 1) / kChunk;
      for (long long ch = 0; ch < nch; ++ch) vw.push_back(make_int2(sidx, (int)ch));
    }
    if (vw.size() >= (size_t)INT32_MAX) { b->err = "vector work list too long"; return bail(PN_ERR_ARG); }
    b->nvwork = (int)vw.size();
    SETUP_B(hipMalloc(&b->vwork, sizeof(int2) * b->nvwork));
    SETUP_B(hipMemcpy(b->vwork, vw.data(), sizeof(int2) * b->nvwork, hipMemcpyHostToDevice));
    b->vfull = std::move(vw);
  }
  b->nlaunch = b->nsys;
  SETUP_B(hipMalloc(&b->active, sizeof(int)));
  SETUP_B(hipHostMalloc(&b->active_host, sizeof(int), hipHostMallocDefault));
  SETUP_B(hipMalloc(&b->flag, sizeof(int)));
  SETUP_B(hipHostMalloc(&b->flag_host, sizeof(int), hipHostMallocDefault));
  SETUP_B(hipStreamSynchronize(b->stream));
#undef SETUP_B
  *out = b;
  return PN_OK;
}

extern "C" pn_status pn_batch_layout(const pn_batch* b, int prob, pn_layout* layout) {
  if (!b || !layout || prob < 0 || prob >= b->nprob) return PN_ERR_ARG;
  return pn_layout_query(b->prob[prob], layout);
}

extern "C" pn_ctx* pn_batch_problem(const pn_batch* b, int prob) {
  if (!b || prob < 0 || prob >= b->nprob) return nullptr;
  return b->prob[prob];
}

extern "C" int pn_batch_zchunk(const pn_batch* b, int prob) {
  if (!b || prob < 0 || prob >= b->nprob) return -1;
  return b->prob[prob]->zchunk;
}

extern "C" long long pn_batch_unknowns(const pn_batch* b) { return b ? b->unknowns : -1; }

extern "C" pn_status pn_batch_bench_apply(pn_batch* b, int iters, int transpose, double* ms_per_apply) {
  if (!b || iters < 1 || !ms_per_apply) return b ? bfail(b, PN_ERR_ARG, "bad arguments") : PN_ERR_ARG;
  hipEvent_t e0, e1;
  B_HIP(hipEventCreate(&e0));
  B_HIP(hipEventCreate(&e1));
  // every system, ungated: y = op(p) into q with the FP64 partial sums
  DevState zero;
  std::memset(&zero, 0, sizeof(zero));
  for (int i = 0; i < b->nsys; ++i) b->st_host[i] = zero;
  B_HIP(hipMemcpyAsync(b->st, b->st_host, sizeof(DevState) * b->nsys, hipMemcpyHostToDevice, b->stream));
  const BatchLaunch bl = roles(b, BV_P, -1, BV_Q, -1, transpose ? -1.0 : 1.0, 0);
  B_HIP(stencil_all(b, K_F32_APPLY, bl, b->stream));  // warm-up
  B_HIP(hipEventRecord(e0, b->stream));
  for (int i = 0; i < iters; ++i) B_HIP(stencil_all(b, K_F32_APPLY, bl, b->stream));
  B_HIP(hipEventRecord(e1, b->stream));
  B_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  B_HIP(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *ms_per_apply = ms / iters;
  return PN_OK;
}

extern "C" pn_status pn_batch_solve(pn_batch* b, const float* const* rhs, double* const* x, double tol,
                                    const pn_solve_opts* opts, pn_solve_info* info) {
  if (!b) return PN_ERR_ARG;
  if (!rhs || !x) return bfail(b, PN_ERR_ARG, "rhs or x is NULL");
  for (int i = 0; i < b->nsys; ++i)
    if (!rhs[i] || !x[i]) return bfail(b, PN_ERR_ARG, "rhs[" + std::to_string(i) + "] or x[...] is NULL");
  if (!(tol > 0.0)) return bfail(b, PN_ERR_ARG, "tol must be > 0");
  pn_solve_opts o;
  pn_default_opts(&o);
  if (opts) o = *opts;
  if (o.max_iter < 1 || o.max_refine < 0 || !(o.inner_tol > 0.0 && o.inner_tol < 1.0))
    return bfail(b, PN_ERR_ARG, "invalid solve options");
  if (o.precision != PN_FP32_IR) return bfail(b, PN_ERR_ARG, "the batched solve runs FP32 with FP64 refinement only");
  if (o.variant < PN_VARIANT_AUTO || o.variant > PN_VARIANT_SCHUR_MG || o.variant == PN_VARIANT_SCHUR)
    return bfail(b, PN_ERR_ARG, "unknown variant");
  const bool mgpath = o.variant == PN_VARIANT_SCHUR_MG;
  if (mgpath)
    for (int p = 0; p < b->nprob; ++p)
      if (!mg_supported(b->prob[p]))
        return bfail(b, PN_ERR_ARG, "problem " + std::to_string(p) + ": the multigrid variant needs no Neumann "
                                    "axis and positive extinction");
  const bool cg = o.variant != PN_VARIANT_CGLS;
  const bool eq = o.variant == PN_VARIANT_AUTO || o.variant == PN_VARIANT_CG_EQ;
  if (info) std::memset(info, 0, sizeof(pn_solve_info) * b->nsys);
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t ss = b->sstream;
  B_HIP(hipEventRecord(b->ev_in, b->stream));
  B_HIP(hipStreamWaitEvent(ss, b->ev_in, 0));
  // non-finite right-hand sides
  B_HIP(hipMemsetAsync(b->flag, 0, sizeof(int), ss));
  for (int i = 0; i < b->nsys; ++i) {
    const long n = b->prob[i / b->nrhs]->n;
    hipLaunchKernelGGL(k_check_finite, dim3(grid_for(n)), dim3(kBlock), 0, ss, rhs[i], n, b->flag);
  }
  B_HIP(hipGetLastError());
  B_HIP(hipMemcpyAsync(b->flag_host, b->flag, sizeof(int), hipMemcpyDeviceToHost, ss));
  B_HIP(hipStreamSynchronize(ss));
  if (*b->flag_host) return bfail(b, PN_ERR_NONFINITE, "a right-hand side contains NaN or Inf");
  // packed -> padded
  for (int i = 0; i < b->nsys; ++i) {
    const pn_ctx* c = b->prob[i / b->nrhs];
    const SysArgs& a = b->sys_h[i];
    B_HIP((launch_pack<float, float, 0>(c, rhs[i], (float*)a.vec[BV_B], ss)));
    if (o.use_guess) {
      B_HIP((launch_pack<double, double, 0>(c, x[i], (double*)a.vec[BV_X64], ss)));
    } else {
      hipLaunchKernelGGL((k_fill<double>), dim3(grid_for(c->nv)), dim3(kBlock), 0, ss, (double*)a.vec[BV_X64],
                         (long)c->nv, 0.0);
      B_HIP(hipGetLastError());
    }
  }
  if (mgpath) {
    // per problem: the first system's scratch vectors serve as the Krylov
    // workspace; every system is solved by the single-system even-parity
    // multigrid path on its own Q and iterate (one captured graph per problem)
    B_HIP(hipStreamSynchronize(ss));
    // problems run concurrently on kMgThreads host threads (each problem has
    // its own solve stream and workspace); largest first to the least-loaded
    // thread.  Every system's arithmetic is independent of the schedule.
    const int hw = (int)std::thread::hardware_concurrency();
    const int nth = std::max(1, std::min(std::min(kMgThreads, b->nprob), hw > 0 ? hw : kMgThreads));
    std::vector<int> order(b->nprob);
    for (int p = 0; p < b->nprob; ++p) order[p] = p;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c2) { return b->prob[a]->n > b->prob[c2]->n; });
    std::vector<std::vector<int>> work(nth);
    std::vector<double> load(nth, 0.0);
    for (int p : order) {
      const int t = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      work[t].push_back(p);
      load[t] += (double)b->prob[p]->n;
    }
    std::vector<pn_status> sstat(b->nsys, PN_OK);
    std::vector<pn_solve_info> sinfo(b->nsys);
    std::vector<std::string> serr(b->nsys);
    // everything that allocates or captures graphs first, on this thread: the
    // worker threads then only launch work on their problems' own streams
    for (int p = 0; p < b->nprob; ++p) {
      pn_ctx* c = b->prob[p];
      pn_status e = borrow_workspace(c, b->sys_h[p * b->nrhs].vec);
      if (e == PN_OK) e = prepare_mg_solve(c, o);
      if (e != PN_OK) {
        const std::string m = pn_last_error(c);
        for (int q = 0; q <= p; ++q) unborrow_workspace(b->prob[q]);
        return bfail(b, e, "problem " + std::to_string(p) + ": " + m);
      }
    }
    int device = 0;
    B_HIP(hipGetDevice(&device));
    auto run = [&](int t) {
      const bool dev_ok = hipSetDevice(device) == hipSuccess;
      for (int p : work[t]) {
        pn_ctx* c = b->prob[p];
        for (int j = 0; j < b->nrhs; ++j) {
          const int i = p * b->nrhs + j;
          if (!dev_ok) { sstat[i] = PN_ERR_HIP; serr[i] = "hipSetDevice failed"; continue; }
          c->b32 = static_cast<float*>(b->sys_h[i].vec[BV_B]);
          c->x64 = static_cast<double*>(b->sys_h[i].vec[BV_X64]);
          sstat[i] = solve_padded_mg(c, tol, o, &sinfo[i]);
          if (sstat[i] != PN_OK) serr[i] = pn_last_error(c);
        }
      }
    };
    std::vector<std::thread> threads;
    for (int t = 1; t < nth; ++t) threads.emplace_back(run, t);
    run(0);
    for (auto& th : threads) th.join();
    for (int p = 0; p < b->nprob; ++p) unborrow_workspace(b->prob[p]);
    pn_status result = PN_OK;
    int first_bad = -1;
    for (int i = 0; i < b->nsys; ++i) {
      if (info) info[i] = sinfo[i];
      if (sstat[i] != PN_OK && first_bad < 0) { first_bad = i; result = sstat[i]; }
    }
    for (int i = 0; i < b->nsys; ++i)
      B_HIP((launch_pack<double, double, 1>(b->prob[i / b->nrhs], (const double*)b->sys_h[i].vec[BV_X64], x[i], ss)));
    B_HIP(hipEventRecord(b->ev_out, ss));
    B_HIP(hipStreamWaitEvent(b->stream, b->ev_out, 0));
    B_HIP(hipStreamSynchronize(ss));
    if (first_bad >= 0)
      bfail(b, result, "system " + std::to_string(first_bad) + ": " + pn_status_string(result) + " (" +
                           serr[first_bad] + ")");
    return result;
  }
  const int gi = o.graph_iters < 2 ? 2 : (o.graph_iters + 1) & ~1;  // even: r ends in r0
  {
    pn_status cs = compact(b, std::vector<char>(b->nsys, 1), ss);
    if (cs != PN_OK) return cs;
  }
  DevState init;
  std::memset(&init, 0, sizeof(init));
  init.max_iters = o.max_iter;
  for (int i = 0; i < b->nsys; ++i) b->st_host[i] = init;
  B_HIP(hipMemcpyAsync(b->st, b->st_host, sizeof(DevState) * b->nsys, hipMemcpyHostToDevice, ss));
  std::vector<int> outer(b->nsys, 0), status(b->nsys, PN_ERR_NOT_CONVERGED);
  std::vector<double> rel(b->nsys, 0.0), bnorm(b->nsys, 0.0);
  for (;;) {
    // r = Q - A x in FP64 for every running system
    B_HIP(stencil_all(b, K_F64_RESID32, roles(b, BV_X64, BV_B, BV_R0, -1, 1.0, 0), ss));
    B_HIP(fin_all<BF_RESID>(b, ss));
    B_HIP(hipMemcpyAsync(b->st_host, b->st, sizeof(DevState) * b->nsys, hipMemcpyDeviceToHost, ss));
    B_HIP(hipStreamSynchronize(ss));
    int nactive = 0;
    for (int i = 0; i < b->nsys; ++i) {
      DevState& h = b->st_host[i];
      if (h.frozen) continue;
      ++outer[i];
      bnorm[i] = std::sqrt(h.bb2);
      int s = -1;
      if (h.bb2 == 0.0) {  // Q = 0: the solution is 0
        const SysArgs& a = b->sys_h[i];
        hipLaunchKernelGGL((k_fill<double>), dim3(grid_for(a.nv)), dim3(kBlock), 0, ss, (double*)a.vec[BV_X64],
                           (long)a.nv, 0.0);
        B_HIP(hipGetLastError());
        rel[i] = 0.0;
        s = PN_OK;
      } else {
        rel[i] = std::sqrt(h.rtrue2 / h.bb2);
        if (info && info[i].nhistory < PN_MAX_HISTORY) info[i].history[info[i].nhistory++] = rel[i];
        if (!std::isfinite(rel[i])) s = PN_ERR_NONFINITE;
        else if (rel[i] <= tol) s = PN_OK;
        else if (outer[i] > o.max_refine || h.iters >= o.max_iter) s = PN_ERR_NOT_CONVERGED;
        else if (h.breakdown) s = PN_ERR_BREAKDOWN;
      }
      if (s >= 0) {
        status[i] = s;
        h.frozen = 1;
      } else {
        // as pn_solve: inner_tol, but no further than the outer tolerance needs
        double itol = std::max(o.inner_tol, 0.3 * tol / rel[i]);
        if (itol >= 1.0) itol = 0.5;
        h.itol2 = itol * itol;
        ++nactive;
      }
    }
    if (nactive == 0) break;
    B_HIP(hipMemcpyAsync(b->st, b->st_host, sizeof(DevState) * b->nsys, hipMemcpyHostToDevice, ss));
    std::vector<char> keep(b->nsys);
    for (int i = 0; i < b->nsys; ++i) keep[i] = b->st_host[i].frozen ? 0 : 1;
    pn_status cs = compact(b, keep, ss);
    if (cs != PN_OK) return cs;
    // inner solves  A d = r0  from d = 0
    B_HIP(vec_all<BO_ZERO_D>(b, ss));
    int rs = BV_R0;
    if (eq) {  // r1 = W r0; the inner solves track <r, W r>
      B_HIP(stencil_all(b, K_F32_EQS, roles(b, BV_R0, -1, BV_R1, -1, 1.0, 0), ss));
      B_HIP(fin_all<BF_RR>(b, ss));
      rs = BV_R1;
    }
    B_HIP(stencil_all(b, K_F32_APPLY, roles(b, rs, -1, BV_S, -1, -1.0, 0), ss));
    B_HIP(fin_all<BF_INIT>(b, ss));
    B_HIP(vec_all<BO_COPY_SP>(b, ss));
    for (;;) {
      if (!b->gexec) {
        pn_status e = build_batch_graph(b, gi, cg, eq);
        if (e != PN_OK) return e;
      }
      B_HIP(hipGraphLaunch(b->gexec, ss));
      hipLaunchKernelGGL(k_batch_active, dim3(1), dim3(kBlock), 0, ss, (const SysArgs*)b->sys, b->nsys, b->active);
      B_HIP(hipGetLastError());
      B_HIP(hipMemcpyAsync(b->active_host, b->active, sizeof(int), hipMemcpyDeviceToHost, ss));
      B_HIP(hipStreamSynchronize(ss));
      const int act = *b->active_host;
      if (act == 0) break;
      if (2 * act <= b->nlaunch) {  // half the launch set finished: launch only the running systems
        B_HIP(hipMemcpyAsync(b->st_host, b->st, sizeof(DevState) * b->nsys, hipMemcpyDeviceToHost, ss));
        B_HIP(hipStreamSynchronize(ss));
        std::vector<char> run(b->nsys);
        for (int i = 0; i < b->nsys; ++i) run[i] = (!b->st_host[i].frozen && !b->st_host[i].done) ? 1 : 0;
        pn_status cs = compact(b, run, ss);
        if (cs != PN_OK) return cs;
      }
    }
    {  // x += d for every system of this refinement step
      pn_status cs = compact(b, keep, ss);
      if (cs != PN_OK) return cs;
    }
    B_HIP(vec_all<BO_AXPY64>(b, ss));
  }
  {
    pn_status cs = compact(b, std::vector<char>(b->nsys, 1), ss);
    if (cs != PN_OK) return cs;
  }
  // padded -> packed (also after a failed solve: x is the last iterate)
  for (int i = 0; i < b->nsys; ++i)
    B_HIP((launch_pack<double, double, 1>(b->prob[i / b->nrhs], (const double*)b->sys_h[i].vec[BV_X64], x[i], ss)));
  B_HIP(hipEventRecord(b->ev_out, ss));
  B_HIP(hipStreamWaitEvent(b->stream, b->ev_out, 0));
  B_HIP(hipStreamSynchronize(ss));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  pn_status result = PN_OK;
  int first_bad = -1;
  for (int i = 0; i < b->nsys; ++i) {
    if (info) {
      info[i].status = status[i];
      info[i].outer_iters = outer[i];
      info[i].inner_iters = b->st_host[i].iters;
      info[i].rel_residual = rel[i];
      info[i].bnorm = bnorm[i];
      info[i].seconds = secs;
      const SolveBytes sb = solve_bytes(b->prob[i / b->nrhs], false, cg, eq);
      info[i].bytes = sb.per_iter * info[i].inner_iters + sb.per_start * std::max(outer[i] - 1, 0) +
                      sb.per_resid * outer[i];
    }
    if (status[i] != PN_OK && first_bad < 0) { first_bad = i; result = (pn_status)status[i]; }
  }
  if (first_bad >= 0)
    bfail(b, result, "system " + std::to_string(first_bad) + ": " + pn_status_string(result));
  return result;
}
