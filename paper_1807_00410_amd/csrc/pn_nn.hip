// C ABI of the learned initial guess / preconditioner network (declarations
// in include/pn_nn.h): the layer primitives and the 4-level U-Net with its
// training step (forward, backward, Adam) on the project's own kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "../../include/pn_nn.h"
#include "pn_nn_kernels.h"

using namespace pn::nn;

namespace {

thread_local std::string g_nn_error;

pn_status nfail(std::string* where, pn_status s, const std::string& m) {
  if (where) *where = m; else g_nn_error = m;
  return s;
}

#define NN_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return nfail(ERRP, e_ == hipErrorOutOfMemory ? PN_ERR_ALLOC : PN_ERR_HIP,           \
                   std::string(#call) + ": " + hipGetErrorString(e_));                    \
  } while (0)

int eblocks(long long n) {
  long long b = (n + kNB - 1) / kNB;
  if (b > 16384) b = 16384;
  return (int)(b < 1 ? 1 : b);
}

bool dims_ok(int B, int nx, int ny, int nz) { return B >= 1 && nx >= 1 && ny >= 1 && nz >= 1; }

Dims mk(int B, int nx, int ny, int nz) {
  Dims d;
  d.B = B; d.D = nz; d.H = ny; d.W = nx;
  d.V = (long long)B * nx * ny * nz;
  return d;
}

Dims half(const Dims& d) { return mk(d.B, d.W / 2, d.H / 2, d.D / 2); }

// --- launches shared by the primitives and the network ---
// persistent convolution blocks: every CU holds two (55 KB of LDS each)
int conv_blocks(const Dims& d) {
  const long long groups = (d.V + 255) / 256;  // 4 waves x 2 tiles x 32 voxels
  return (int)(groups < 512 ? (groups < 1 ? 1 : groups) : 512);
}

hipError_t conv_fwd(const Dims& d, const uint16_t* x, const uint16_t* w, const float* bias, bool relu, bool f32,
                    void* y, hipStream_t s) {
  const int nb = conv_blocks(d);
  if (f32) {
    if (relu) hipLaunchKernelGGL((k_conv3d<false, true, true>), dim3(nb), dim3(kNB), 0, s, x, w, bias, y, d);
    else hipLaunchKernelGGL((k_conv3d<false, false, true>), dim3(nb), dim3(kNB), 0, s, x, w, bias, y, d);
  } else {
    if (relu) hipLaunchKernelGGL((k_conv3d<false, true, false>), dim3(nb), dim3(kNB), 0, s, x, w, bias, y, d);
    else hipLaunchKernelGGL((k_conv3d<false, false, false>), dim3(nb), dim3(kNB), 0, s, x, w, bias, y, d);
  }
  return hipGetLastError();
}

hipError_t conv_dgrad(const Dims& d, const uint16_t* g, const uint16_t* w, uint16_t* dx, hipStream_t s) {
  const int nb = conv_blocks(d);
  hipLaunchKernelGGL((k_conv3d<true, false, false>), dim3(nb), dim3(kNB), 0, s, g, w, (const float*)nullptr,
                     (void*)dx, d);
  return hipGetLastError();
}

// block count and voxels per block of the weight-gradient kernel
void wgrad_split(const Dims& d, int* nblk, long long* per) {
  long long nb = (d.V + 255) / 256;
  if (nb > 512) nb = 512;
  if (nb < 1) nb = 1;
  long long p = (d.V + nb - 1) / nb;
  p = (p + 15) / 16 * 16;
  *per = p;
  *nblk = (int)((d.V + p - 1) / p);
}

hipError_t conv_wgrad(const Dims& d, const uint16_t* x, const uint16_t* g, float* dw, float* db, float* wpart,
                      float* bpart, hipStream_t s) {
  int nblk;
  long long per;
  wgrad_split(d, &nblk, &per);
  hipLaunchKernelGGL(k_conv3d_wgrad, dim3(nblk), dim3(kNB), 0, s, x, g, wpart, bpart, d, per);
  hipLaunchKernelGGL(k_reduce_parts, dim3((kWElems + kNB - 1) / kNB), dim3(kNB), 0, s, (const float*)wpart, nblk,
                     kWElems, dw);
  hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(kNB), 0, s, (const float*)bpart, nblk, kC, db);
  return hipGetLastError();
}

}  // namespace

// =================================================================== net ==
static constexpr int kConv = 15;
static constexpr long long kPer = kWElems + kC;  // parameters per convolution
static constexpr long long kNParams = kConv * kPer;

struct pn_net {
  hipStream_t stream = nullptr;
  float* p = nullptr;   // FP32 master parameters [15][27648 w + 32 b]
  float* g = nullptr;   // gradients, same layout
  float* m = nullptr;   // Adam moments
  float* v = nullptr;
  uint16_t* wb = nullptr;  // bfloat16 weights [15][27648]
  long long step = 0;
  // activation / gradient buffers of the current shape
  int B = 0, nx = 0, ny = 0, nz = 0;
  std::vector<void*> owned;
  uint16_t* a[4][8] = {};   // per level: activations (see forward)
  uint16_t* gr[4][3] = {};  // per level: two working gradients and the skip gradient
  float* y = nullptr;       // FP32 output [V0][32]
  float* wpart = nullptr;
  float* bpart = nullptr;
  double* lpart = nullptr;
  double* lpart_host = nullptr;
  std::string err;
};

#define ERRP (&n->err)

namespace {

float* wf(pn_net* n, int i) { return n->p + i * kPer; }
float* bf(pn_net* n, int i) { return n->p + i * kPer + kWElems; }
float* gw(pn_net* n, int i) { return n->g + i * kPer; }
float* gb(pn_net* n, int i) { return n->g + i * kPer + kWElems; }
const uint16_t* wb(pn_net* n, int i) { return n->wb + (long long)i * kWElems; }

void free_shape(pn_net* n) {
  for (void* q : n->owned) hipFree(q);
  n->owned.clear();
  std::memset(n->a, 0, sizeof(n->a));
  std::memset(n->gr, 0, sizeof(n->gr));
  n->y = nullptr; n->wpart = nullptr; n->bpart = nullptr; n->lpart = nullptr;
  if (n->lpart_host) { hipHostFree(n->lpart_host); n->lpart_host = nullptr; }
  n->B = n->nx = n->ny = n->nz = 0;
}

// Level-l activation slots: 0 pool output / input copy, 1 first conv, 2 second
// conv (skip), 3 decoder input (up + skip), 4 first decoder conv, 5 second.
pn_status ensure_shape(pn_net* n, int B, int nx, int ny, int nz) {
  if (n->B == B && n->nx == nx && n->ny == ny && n->nz == nz) return PN_OK;
  free_shape(n);
  Dims d = mk(B, nx, ny, nz);
  auto alloc = [&](size_t bytes, void** out) -> hipError_t {
    hipError_t e = hipMalloc(out, bytes);
    if (e == hipSuccess) n->owned.push_back(*out);
    return e;
  };
  for (int l = 0; l < 4; ++l) {
    const size_t bytes = (size_t)d.V * kC * sizeof(uint16_t);
    for (int s = 0; s < 6; ++s) NN_HIP(alloc(bytes, (void**)&n->a[l][s]));
    for (int s = 0; s < 3; ++s) NN_HIP(alloc(bytes, (void**)&n->gr[l][s]));
    d = half(d);
  }
  Dims d0 = mk(B, nx, ny, nz);
  NN_HIP(alloc((size_t)d0.V * kC * sizeof(float), (void**)&n->y));
  NN_HIP(alloc((size_t)512 * kWElems * sizeof(float), (void**)&n->wpart));
  NN_HIP(alloc((size_t)512 * kC * sizeof(float), (void**)&n->bpart));
  NN_HIP(alloc((size_t)4096 * sizeof(double), (void**)&n->lpart));
  NN_HIP(hipHostMalloc((void**)&n->lpart_host, 4096 * sizeof(double), hipHostMallocDefault));
  n->B = B; n->nx = nx; n->ny = ny; n->nz = nz;
  return PN_OK;
}

// conv index i at level l: encoder 2l, 2l+1 (l < 4); decoder level l (0..2): 12-2l, 13-2l
pn_status forward(pn_net* n, const uint16_t* x, hipStream_t s) {
  Dims d[4];
  d[0] = mk(n->B, n->nx, n->ny, n->nz);
  for (int l = 1; l < 4; ++l) d[l] = half(d[l - 1]);
  // encoder
  const uint16_t* in = x;
  for (int l = 0; l < 4; ++l) {
    if (l > 0) {
      hipLaunchKernelGGL(k_pool2, dim3(eblocks(d[l].V * kC)), dim3(kNB), 0, s, (const uint16_t*)n->a[l - 1][2],
                         n->a[l][0], d[l]);
      in = n->a[l][0];
    }
    NN_HIP(conv_fwd(d[l], in, wb(n, 2 * l), bf(n, 2 * l), true, false, n->a[l][1], s));
    NN_HIP(conv_fwd(d[l], n->a[l][1], wb(n, 2 * l + 1), bf(n, 2 * l + 1), true, false, n->a[l][2], s));
  }
  // decoder: level 3 output is a[3][2]
  const uint16_t* below = n->a[3][2];
  for (int l = 2; l >= 0; --l) {
    const int c0 = 12 - 2 * l;
    hipLaunchKernelGGL(k_up2_add, dim3(eblocks(d[l].V * kC)), dim3(kNB), 0, s, below, (const uint16_t*)n->a[l][2],
                       n->a[l][3], d[l]);
    NN_HIP(conv_fwd(d[l], n->a[l][3], wb(n, c0), bf(n, c0), true, false, n->a[l][4], s));
    NN_HIP(conv_fwd(d[l], n->a[l][4], wb(n, c0 + 1), bf(n, c0 + 1), true, false, n->a[l][5], s));
    below = n->a[l][5];
  }
  NN_HIP(conv_fwd(d[0], n->a[0][5], wb(n, 14), bf(n, 14), false, true, n->y, s));
  return PN_OK;
}

// Backward of one conv with ReLU output `out`: g (gradient wrt out, masked in
// place), weight gradient from its input, input gradient into gin (may be null).
pn_status conv_back(pn_net* n, int i, const Dims& d, uint16_t* g, const uint16_t* out, const uint16_t* in,
                    uint16_t* gin, hipStream_t s) {
  if (out) hipLaunchKernelGGL(k_relu_mask, dim3(eblocks(d.V * kC)), dim3(kNB), 0, s, g, out, d.V * kC);
  NN_HIP(conv_wgrad(d, in, g, gw(n, i), gb(n, i), n->wpart, n->bpart, s));
  if (gin) NN_HIP(conv_dgrad(d, g, wb(n, i), gin, s));
  return PN_OK;
}

pn_status backward(pn_net* n, const uint16_t* x, const uint16_t* g_out, hipStream_t s) {
  Dims d[4];
  d[0] = mk(n->B, n->nx, n->ny, n->nz);
  for (int l = 1; l < 4; ++l) d[l] = half(d[l - 1]);
  pn_status e;
  // output conv: gradient wrt a[0][5] into gr[0][0]
  if ((e = conv_back(n, 14, d[0], const_cast<uint16_t*>(g_out), nullptr, n->a[0][5], n->gr[0][0], s)) != PN_OK) return e;
  // decoder levels 0, 1, 2: gr[l][0] holds the gradient wrt a[l][5]
  for (int l = 0; l <= 2; ++l) {
    const int c0 = 12 - 2 * l;
    if ((e = conv_back(n, c0 + 1, d[l], n->gr[l][0], n->a[l][5], n->a[l][4], n->gr[l][1], s)) != PN_OK) return e;
    if ((e = conv_back(n, c0, d[l], n->gr[l][1], n->a[l][4], n->a[l][3], n->gr[l][2], s)) != PN_OK) return e;
    // gr[l][2]: gradient wrt the decoder input (kept for the skip); up2 adjoint -> level l+1
    hipLaunchKernelGGL(k_up2_bwd, dim3(eblocks(d[l + 1].V * kC)), dim3(kNB), 0, s, (const uint16_t*)n->gr[l][2],
                       n->gr[l + 1][0], d[l + 1]);
  }
  // bottleneck and encoder, level 3 .. 0: gr[l][0] holds the gradient wrt a[l][2]
  for (int l = 3; l >= 0; --l) {
    const uint16_t* in0 = l > 0 ? n->a[l][0] : x;
    if ((e = conv_back(n, 2 * l + 1, d[l], n->gr[l][0], n->a[l][2], n->a[l][1], n->gr[l][1], s)) != PN_OK) return e;
    if ((e = conv_back(n, 2 * l, d[l], n->gr[l][1], n->a[l][1], in0, l > 0 ? n->gr[l][0] : nullptr, s)) != PN_OK)
      return e;
    if (l > 0) {  // pool adjoint plus the skip gradient of level l-1
      hipLaunchKernelGGL(k_pool2_bwd_add, dim3(eblocks(d[l - 1].V * kC)), dim3(kNB), 0, s,
                         (const uint16_t*)n->gr[l][0], (const uint16_t*)n->gr[l - 1][2], n->gr[l - 1][0], d[l - 1]);
    }
  }
  NN_HIP(hipGetLastError());
  return PN_OK;
}

pn_status repack(pn_net* n) {
  hipLaunchKernelGGL(k_pack_weights, dim3(eblocks(kConv * kWElems)), dim3(kNB), 0, n->stream, (const float*)n->p,
                     n->wb, kConv);
  NN_HIP(hipGetLastError());
  return PN_OK;
}

}  // namespace

#undef ERRP
#define ERRP (n ? &n->err : nullptr)

extern "C" int pn_net_nparams(void) { return (int)kNParams; }

extern "C" const char* pn_net_last_error(const pn_net* n) { return n ? n->err.c_str() : g_nn_error.c_str(); }

extern "C" void pn_net_destroy(pn_net* n) {
  if (!n) return;
  if (n->stream) hipStreamSynchronize(n->stream);
  free_shape(n);
  hipFree(n->p); hipFree(n->g); hipFree(n->m); hipFree(n->v); hipFree(n->wb);
  delete n;
}

extern "C" pn_status pn_net_create(unsigned long long seed, void* stream, pn_net** out) {
  if (!out) return nfail(nullptr, PN_ERR_ARG, "out is NULL");
  *out = nullptr;
  pn_net* n = new pn_net();
  n->stream = (hipStream_t)stream;
  auto bail = [&](pn_status s) {
    std::string m = n->err;
    pn_net_destroy(n);
    return nfail(nullptr, s, m);
  };
#define C_HIP(call)                                                                                   \
  do {                                                                                                \
    hipError_t e_ = (call);                                                                           \
    if (e_ != hipSuccess) {                                                                           \
      n->err = std::string(#call) + ": " + hipGetErrorString(e_);                                     \
      return bail(e_ == hipErrorOutOfMemory ? PN_ERR_ALLOC : PN_ERR_HIP);                             \
    }                                                                                                 \
  } while (0)
  C_HIP(hipMalloc(&n->p, sizeof(float) * kNParams));
  C_HIP(hipMalloc(&n->g, sizeof(float) * kNParams));
  C_HIP(hipMalloc(&n->m, sizeof(float) * kNParams));
  C_HIP(hipMalloc(&n->v, sizeof(float) * kNParams));
  C_HIP(hipMalloc(&n->wb, sizeof(uint16_t) * kConv * kWElems));
  // He-normal weights (output convolution scaled by 0.1), zero biases
  std::vector<float> h(kNParams, 0.f);
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  const double sd = std::sqrt(2.0 / (kTaps * kC));
  for (int i = 0; i < kConv; ++i)
    for (int e = 0; e < kWElems; ++e) h[i * kPer + e] = (float)(nd(rng) * sd * (i == kConv - 1 ? 0.1 : 1.0));
  C_HIP(hipMemcpy(n->p, h.data(), sizeof(float) * kNParams, hipMemcpyHostToDevice));
  C_HIP(hipMemset(n->g, 0, sizeof(float) * kNParams));
  C_HIP(hipMemset(n->m, 0, sizeof(float) * kNParams));
  C_HIP(hipMemset(n->v, 0, sizeof(float) * kNParams));
#undef C_HIP
  if (repack(n) != PN_OK) return bail(PN_ERR_HIP);
  *out = n;
  return PN_OK;
}

extern "C" void* pn_net_get_stream(const pn_net* n) { return n ? (void*)n->stream : nullptr; }

extern "C" pn_status pn_net_set_stream(pn_net* n, void* stream) {
  if (!n) return nfail(nullptr, PN_ERR_ARG, "net is NULL");
  n->stream = (hipStream_t)stream;
  return PN_OK;
}

extern "C" pn_status pn_net_get_params(pn_net* n, float* host, float* host_grads) {
  if (!n || (!host && !host_grads)) return nfail(ERRP, PN_ERR_ARG, "bad arguments");
  NN_HIP(hipStreamSynchronize(n->stream));
  if (host) NN_HIP(hipMemcpy(host, n->p, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
  if (host_grads) NN_HIP(hipMemcpy(host_grads, n->g, sizeof(float) * kNParams, hipMemcpyDeviceToHost));
  return PN_OK;
}

extern "C" pn_status pn_net_set_params(pn_net* n, const float* host) {
  if (!n || !host) return nfail(ERRP, PN_ERR_ARG, "bad arguments");
  for (long long i = 0; i < kNParams; ++i)
    if (!std::isfinite(host[i])) return nfail(ERRP, PN_ERR_NONFINITE, "non-finite parameter");
  NN_HIP(hipStreamSynchronize(n->stream));
  NN_HIP(hipMemcpy(n->p, host, sizeof(float) * kNParams, hipMemcpyHostToDevice));
  NN_HIP(hipMemset(n->m, 0, sizeof(float) * kNParams));
  NN_HIP(hipMemset(n->v, 0, sizeof(float) * kNParams));
  n->step = 0;
  return repack(n);
}

static const char kMagic[8] = {'P', 'N', 'U', 'N', 'E', 'T', '0', '1'};

extern "C" pn_status pn_net_save(pn_net* n, const char* path) {
  if (!n || !path) return nfail(ERRP, PN_ERR_ARG, "bad arguments");
  std::vector<float> h(kNParams);
  pn_status s = pn_net_get_params(n, h.data(), nullptr);
  if (s != PN_OK) return s;
  FILE* f = std::fopen(path, "wb");
  if (!f) return nfail(ERRP, PN_ERR_ARG, std::string("cannot write ") + path);
  const long long np = kNParams;
  bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&np, sizeof(np), 1, f) == 1 &&
            std::fwrite(&n->step, sizeof(n->step), 1, f) == 1 &&
            std::fwrite(h.data(), sizeof(float), kNParams, f) == (size_t)kNParams;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? PN_OK : nfail(ERRP, PN_ERR_ARG, std::string("short write to ") + path);
}

extern "C" pn_status pn_net_load(pn_net* n, const char* path) {
  if (!n || !path) return nfail(ERRP, PN_ERR_ARG, "bad arguments");
  FILE* f = std::fopen(path, "rb");
  if (!f) return nfail(ERRP, PN_ERR_ARG, std::string("cannot read ") + path);
  char magic[8];
  long long np = 0, step = 0;
  std::vector<float> h(kNParams);
  const bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 &&
                  std::fread(&np, sizeof(np), 1, f) == 1 && np == kNParams &&
                  std::fread(&step, sizeof(step), 1, f) == 1 &&
                  std::fread(h.data(), sizeof(float), kNParams, f) == (size_t)kNParams;
  std::fclose(f);
  if (!ok) return nfail(ERRP, PN_ERR_ARG, std::string("not a network file of this layout: ") + path);
  pn_status s = pn_net_set_params(n, h.data());
  n->step = step;
  return s;
}

static bool net_dims_ok(int B, int nx, int ny, int nz) {
  return dims_ok(B, nx, ny, nz) && nx % 8 == 0 && ny % 8 == 0 && nz % 8 == 0 &&
         (long long)B * nx * ny * nz <= (1LL << 27);
}

extern "C" pn_status pn_net_forward(pn_net* n, int B, int nx, int ny, int nz, const uint16_t* x, float* y) {
  if (!n || !x || !y) return nfail(ERRP, PN_ERR_ARG, "bad arguments");
  if (!net_dims_ok(B, nx, ny, nz)) return nfail(ERRP, PN_ERR_ARG, "extents must be positive multiples of 8");
  pn_status s = ensure_shape(n, B, nx, ny, nz);
  if (s != PN_OK) return s;
  if ((s = forward(n, x, n->stream)) != PN_OK) return s;
  const long long V = (long long)B * nx * ny * nz;
  NN_HIP(hipMemcpyAsync(y, n->y, sizeof(float) * V * kC, hipMemcpyDeviceToDevice, n->stream));
  return PN_OK;
}

extern "C" pn_status pn_net_train_step(pn_net* n, int B, int nx, int ny, int nz, const uint16_t* x,
                                       const uint16_t* target, int nout, float lr, double* loss) {
  if (!n || !x || !target) return nfail(ERRP, PN_ERR_ARG, "bad arguments");
  if (!net_dims_ok(B, nx, ny, nz)) return nfail(ERRP, PN_ERR_ARG, "extents must be positive multiples of 8");
  if (nout < 1 || nout > kC || !(lr >= 0.f)) return nfail(ERRP, PN_ERR_ARG, "nout in 1..32, lr >= 0");
  pn_status s = ensure_shape(n, B, nx, ny, nz);
  if (s != PN_OK) return s;
  hipStream_t st = n->stream;
  if ((s = forward(n, x, st)) != PN_OK) return s;
  const long long V = (long long)B * nx * ny * nz;
  const int nb = std::min(eblocks(V * kC), 4096);
  // output gradient into gr[1][2] of level 0's spare slot: use a[0][0] (unused at level 0)
  uint16_t* gout = n->a[0][0];
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(kNB), 0, st, (const float*)n->y, target, gout, V, nout,
                     1.0 / ((double)V * nout), n->lpart);
  NN_HIP(hipGetLastError());
  NN_HIP(hipMemcpyAsync(n->lpart_host, n->lpart, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
  if ((s = backward(n, x, gout, st)) != PN_OK) return s;
  if (lr > 0.f) {
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)n->step));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)n->step));
    hipLaunchKernelGGL(k_adam, dim3(eblocks(kNParams)), dim3(kNB), 0, st, n->p, (const float*)n->g, n->m, n->v,
                       kNParams, lr, b1, (float)(1.0 - 0.9), b2, (float)(1.0 - 0.999), 1e-8f, bc1, bc2);
    NN_HIP(hipGetLastError());
    if ((s = repack(n)) != PN_OK) return s;
  }
  NN_HIP(hipStreamSynchronize(st));
  double sum = 0.0;
  for (int i = 0; i < nb; ++i) sum += n->lpart_host[i];
  if (loss) *loss = sum / ((double)V * nout);
  return std::isfinite(sum) ? PN_OK : nfail(ERRP, PN_ERR_NONFINITE, "non-finite loss");
}

// Training loop over samples held as separate device tensors: each epoch
// visits the samples in a seeded random order, gathers `batch` of them into
// contiguous staging buffers and takes one training step with a cosine-decayed
// learning rate.  *loss_out: mean loss of the last epoch.
extern "C" pn_status pn_net_train(pn_net* n, int nsamples, int nx, int ny, int nz, const uint16_t* const* x,
                                  const uint16_t* const* t, int nout, int epochs, int batch, float lr,
                                  unsigned long long seed, double* loss_out) {
  if (!n || !x || !t || nsamples < 1 || epochs < 1 || batch < 1 || batch > nsamples || !(lr > 0.f))
    return nfail(ERRP, PN_ERR_ARG, "bad arguments");
  if (!net_dims_ok(batch, nx, ny, nz) || nout < 1 || nout > kC)
    return nfail(ERRP, PN_ERR_ARG, "extents must be positive multiples of 8, nout in 1..32");
  for (int i = 0; i < nsamples; ++i)
    if (!x[i] || !t[i]) return nfail(ERRP, PN_ERR_ARG, "a sample pointer is NULL");
  const size_t vx = (size_t)nx * ny * nz * kC, vt = (size_t)nx * ny * nz * nout;
  uint16_t *bx = nullptr, *bt = nullptr;
  NN_HIP(hipMalloc(&bx, sizeof(uint16_t) * vx * batch));
  hipError_t he = hipMalloc(&bt, sizeof(uint16_t) * vt * batch);
  if (he != hipSuccess) { hipFree(bx); NN_HIP(he); }
  std::mt19937_64 rng(seed);
  std::vector<int> order(nsamples);
  for (int i = 0; i < nsamples; ++i) order[i] = i;
  const int steps_per_epoch = nsamples / batch;
  const long long total = (long long)epochs * steps_per_epoch;
  long long step = 0;
  pn_status st = PN_OK;
  double last = 0.0;
  for (int ep = 0; ep < epochs && st == PN_OK; ++ep) {
    std::shuffle(order.begin(), order.end(), rng);
    double sum = 0.0;
    for (int b = 0; b < steps_per_epoch && st == PN_OK; ++b) {
      for (int j = 0; j < batch; ++j) {
        const int i = order[b * batch + j];
        if (hipMemcpyAsync(bx + vx * j, x[i], sizeof(uint16_t) * vx, hipMemcpyDeviceToDevice, n->stream) != hipSuccess ||
            hipMemcpyAsync(bt + vt * j, t[i], sizeof(uint16_t) * vt, hipMemcpyDeviceToDevice, n->stream) != hipSuccess)
          st = nfail(ERRP, PN_ERR_HIP, "staging copy failed");
      }
      if (st != PN_OK) break;
      const float lr_t = (float)(0.5 * lr * (1.0 + std::cos(3.14159265358979323846 * (double)step / (double)total)));
      double loss = 0.0;
      st = pn_net_train_step(n, batch, nx, ny, nz, bx, bt, nout, lr_t, &loss);
      sum += loss;
      ++step;
    }
    last = sum / steps_per_epoch;
  }
  hipFree(bx);
  hipFree(bt);
  if (st == PN_OK && loss_out) *loss_out = last;
  return st;
}

#undef ERRP
#define ERRP nullptr

// ============================================================ primitives ==
extern "C" pn_status pn_nn_conv3d(int B, int nx, int ny, int nz, const uint16_t* x, const uint16_t* w,
                                  const float* bias, int relu, int out_f32, void* y, void* stream) {
  if (!dims_ok(B, nx, ny, nz) || !x || !w || !y) return nfail(nullptr, PN_ERR_ARG, "bad arguments");
  NN_HIP(conv_fwd(mk(B, nx, ny, nz), x, w, bias, relu != 0, out_f32 != 0, y, (hipStream_t)stream));
  return PN_OK;
}

extern "C" pn_status pn_nn_conv3d_dgrad(int B, int nx, int ny, int nz, const uint16_t* g, const uint16_t* w,
                                        uint16_t* dx, void* stream) {
  if (!dims_ok(B, nx, ny, nz) || !g || !w || !dx) return nfail(nullptr, PN_ERR_ARG, "bad arguments");
  NN_HIP(conv_dgrad(mk(B, nx, ny, nz), g, w, dx, (hipStream_t)stream));
  return PN_OK;
}

extern "C" pn_status pn_nn_conv3d_wgrad(int B, int nx, int ny, int nz, const uint16_t* x, const uint16_t* g,
                                        float* dw, float* db, void* stream) {
  if (!dims_ok(B, nx, ny, nz) || !x || !g || !dw || !db) return nfail(nullptr, PN_ERR_ARG, "bad arguments");
  const Dims d = mk(B, nx, ny, nz);
  int nblk;
  long long per;
  wgrad_split(d, &nblk, &per);
  float *wp = nullptr, *bp = nullptr;
  hipStream_t s = (hipStream_t)stream;
  NN_HIP(hipMalloc(&wp, sizeof(float) * (size_t)nblk * kWElems));
  hipError_t e = hipMalloc(&bp, sizeof(float) * (size_t)nblk * kC);
  if (e == hipSuccess) e = conv_wgrad(d, x, g, dw, db, wp, bp, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(wp);
  hipFree(bp);
  NN_HIP(e);
  return PN_OK;
}

// ------------------------------------------- allocation-free weight gradient --
// The per-block partial sums of the weight gradient live in a file-scope
// device array instead of a temporary allocation.  Each device holds its own
// copy; its address is taken once per device with hipGetSymbolAddress (the
// array's name in host code is not a device address).  Every call on a device
// shares that device's copy: calls that overlap on one device race.
namespace {
constexpr int kWgradScratchBlocks = 128;
constexpr long long kWgradScratchFloats = (long long)kWgradScratchBlocks * (kWElems + kC);
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) float scratch[kWgradScratchFloats];

static float* g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

// Device address of this device's scratch array (taken on first use).
static hipError_t scratch_address(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

extern "C" pn_status pn_nn_conv3d_wgrad_noalloc(int B, int nx, int ny, int nz, const uint16_t* x,
                                                const uint16_t* g, float* dw, float* db, void* stream) {
  if (!dims_ok(B, nx, ny, nz) || !x || !g || !dw || !db) return nfail(nullptr, PN_ERR_ARG, "bad arguments");
  const Dims d = mk(B, nx, ny, nz);
  int nblk;
  long long per;
  wgrad_split(d, &nblk, &per);
  if (nblk > kWgradScratchBlocks)
    return nfail(nullptr, PN_ERR_ARG,
                 "volume of " + std::to_string(d.V) + " voxels needs " + std::to_string(nblk) +
                     " partial-sum blocks; the allocation-free weight gradient holds at most " +
                     std::to_string(kWgradScratchBlocks) + " (B*nx*ny*nz <= " +
                     std::to_string(kWgradScratchBlocks * 256) + ")");
  float* sp = nullptr;
  NN_HIP(scratch_address(&sp));
  // every partial of blocks [0, nblk) is written by the weight-gradient
  // kernel before the reduction reads it: nothing to clear
  NN_HIP(conv_wgrad(d, x, g, dw, db, sp, sp + (long long)kWgradScratchBlocks * kWElems, (hipStream_t)stream));
  return PN_OK;
}

extern "C" pn_status pn_nn_pool2(int B, int nx, int ny, int nz, const uint16_t* x, uint16_t* y, void* stream) {
  if (!dims_ok(B, nx, ny, nz) || nx % 2 || ny % 2 || nz % 2 || !x || !y) return nfail(nullptr, PN_ERR_ARG, "bad arguments");
  const Dims dc = mk(B, nx / 2, ny / 2, nz / 2);
  hipLaunchKernelGGL(k_pool2, dim3(eblocks(dc.V * kC)), dim3(kNB), 0, (hipStream_t)stream, x, y, dc);
  NN_HIP(hipGetLastError());
  return PN_OK;
}

extern "C" pn_status pn_nn_pool2_bwd_add(int B, int nx, int ny, int nz, const uint16_t* gc, const uint16_t* skip,
                                         uint16_t* gf, void* stream) {
  if (!dims_ok(B, nx, ny, nz) || nx % 2 || ny % 2 || nz % 2 || !gc || !gf) return nfail(nullptr, PN_ERR_ARG, "bad arguments");
  const Dims df = mk(B, nx, ny, nz);
  hipLaunchKernelGGL(k_pool2_bwd_add, dim3(eblocks(df.V * kC)), dim3(kNB), 0, (hipStream_t)stream, gc, skip, gf, df);
  NN_HIP(hipGetLastError());
  return PN_OK;
}

extern "C" pn_status pn_nn_up2_add(int B, int nx, int ny, int nz, const uint16_t* xc, const uint16_t* skip,
                                   uint16_t* y, void* stream) {
  if (!dims_ok(B, nx, ny, nz) || nx % 2 || ny % 2 || nz % 2 || !xc || !y) return nfail(nullptr, PN_ERR_ARG, "bad arguments");
  const Dims df = mk(B, nx, ny, nz);
  hipLaunchKernelGGL(k_up2_add, dim3(eblocks(df.V * kC)), dim3(kNB), 0, (hipStream_t)stream, xc, skip, y, df);
  NN_HIP(hipGetLastError());
  return PN_OK;
}

extern "C" pn_status pn_nn_up2_bwd(int B, int nx, int ny, int nz, const uint16_t* gf, uint16_t* gc, void* stream) {
  if (!dims_ok(B, nx, ny, nz) || nx % 2 || ny % 2 || nz % 2 || !gf || !gc) return nfail(nullptr, PN_ERR_ARG, "bad arguments");
  const Dims dc = mk(B, nx / 2, ny / 2, nz / 2);
  hipLaunchKernelGGL(k_up2_bwd, dim3(eblocks(dc.V * kC)), dim3(kNB), 0, (hipStream_t)stream, gf, gc, dc);
  NN_HIP(hipGetLastError());
  return PN_OK;
}

extern "C" pn_status pn_nn_adam(float* w, const float* g, float* m, float* v, long long n, long long step, float lr,
                                double beta1, double beta2, float eps, void* stream) {
  if (!w || !g || !m || !v || n < 1 || step < 1) return nfail(nullptr, PN_ERR_ARG, "bad arguments");
  const float bc1 = (float)(1.0 - std::pow(beta1, (double)step));
  const float bc2 = (float)(1.0 - std::pow(beta2, (double)step));
  hipLaunchKernelGGL(k_adam, dim3(eblocks(n)), dim3(kNB), 0, (hipStream_t)stream, w, g, m, v, n, lr, (float)beta1,
                     (float)(1.0 - beta1), (float)beta2, (float)(1.0 - beta2), eps, bc1, bc2);
  NN_HIP(hipGetLastError());
  return PN_OK;
}

extern "C" const char* pn_nn_last_error(void) { return g_nn_error.c_str(); }
