// HIP kernels of the learned initial guess / preconditioner (gfx950).
//
// Tensors are channels-last bfloat16: t[b][z][y][x][c] with kC = 32 channels
// (64 bytes per voxel), voxels flattened in (b, z, y, x) order.  Every
// convolution is 3x3x3, kC -> kC, zero padded; weights w[t][co][ci] with tap
// t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1).
//
// Convolution as an implicit GEMM on the matrix cores: per tap, the
// [voxels x ci] slab of the shifted input times the [ci x co] weight slice,
// accumulated over the 27 taps in FP32 with v_mfma_f32_32x32x16_bf16 (M = 32
// voxels, N = 32 output channels, K = 16 input channels per instruction).  A
// wave owns two 32-voxel tiles so every weight fragment read from LDS feeds
// two MFMAs; the blocks are persistent (two per CU, the LDS bound) and stage
// the 55 KB weight tensor in LDS once, then loop over voxel tiles; the tap
// loop is unrolled by three (four tiles per wave, or all 27 taps unrolled --
// 256 VGPRs, one wave per SIMD -- were measured slower).
// The input gradient is the same kernel on the flipped, transposed weights
// (the flip is done while filling LDS).  The weight gradient contracts over
// voxels: D[co][ci] = sum_v g[v][co] x[v + d_t][ci], again on MFMA with K = 16
// voxels per instruction, each wave owning a subset of the taps and each
// block a range of voxels; block partials are reduced in a fixed order.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pn {
namespace nn {

constexpr int kC = 32;
constexpr int kTaps = 27;
constexpr int kWElems = kTaps * kC * kC;  // 27648
constexpr int kNB = 256;                  // threads per block

typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// float -> bfloat16, round to nearest even (inputs are finite)
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ bf16x8 as_bf8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

struct Dims {
  int B, D, H, W;
  long long V;  // B*D*H*W
};

__device__ __forceinline__ void decompose(long long v, const Dims& d, int& b, int& z, int& y, int& x) {
  x = (int)(v % d.W);
  long long r = v / d.W;
  y = (int)(r % d.H);
  r /= d.H;
  z = (int)(r % d.D);
  b = (int)(r / d.D);
}

// ------------------------------------------------------------ convolution --
// FLIP = false: Y = conv(X, w) (+ bias, ReLU), weights [t][co][ci].
// FLIP = true:  Y = conv^T(X, w) (input gradient): uses w'[t][ci][co] = w[26-t][co][ci].
// OUTF32: FP32 output, else bfloat16.
constexpr int kMT = 2;  // 32-voxel tiles per wave

template <bool FLIP, bool RELU, bool OUTF32>
__global__ void __launch_bounds__(kNB) k_conv3d(const uint16_t* __restrict__ X, const uint16_t* __restrict__ Wg,
                                                const float* __restrict__ bias, void* __restrict__ Yv, const Dims d) {
  __shared__ uint4 lw4[kWElems / 8];  // [t][n][k], k contiguous (55296 bytes)
  uint16_t* lw = reinterpret_cast<uint16_t*>(lw4);
  if constexpr (!FLIP) {
    const uint4* src = reinterpret_cast<const uint4*>(Wg);
    for (int i = threadIdx.x; i < kWElems / 8; i += kNB) lw4[i] = src[i];
  } else {
    // n (= ci of w) fastest over the threads: the reads of w are contiguous
    for (int i = threadIdx.x; i < kWElems; i += kNB) {
      const int t = i / (kC * kC), k = (i / kC) % kC, n = i % kC;  // n: output = ci of w, k: input = co of w
      lw[(t * kC + n) * kC + k] = Wg[((kTaps - 1 - t) * kC + k) * kC + n];
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row = lane & 31, half = lane >> 5;
  const long long HW = (long long)d.H * d.W;
  const float bj = bias ? bias[row] : 0.f;
  // persistent blocks: the weights are staged once, then groups of
  // (4 waves x kMT tiles x 32 voxels) are taken in turn
  const long long ngroups = (d.V + 32 * kMT * (kNB / 64) - 1) / (32 * kMT * (kNB / 64));
  for (long long grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const long long tile0 = (grp * (kNB / 64) + wv) * kMT;
    int zz[kMT], yy[kMT], xx[kMT];
    long long vv[kMT];
#pragma unroll
    for (int m = 0; m < kMT; ++m) {
      vv[m] = (tile0 + m) * 32 + row;
      int b;
      if (vv[m] < d.V) {
        decompose(vv[m], d, b, zz[m], yy[m], xx[m]);
      } else {
        zz[m] = -4; yy[m] = 0; xx[m] = 0;  // fails every bounds test
      }
    }
    f32x16 acc[kMT];
#pragma unroll
    for (int m = 0; m < kMT; ++m)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[m][r] = 0.f;

    // taps unrolled by three (one x row of the stencil): the loads of a row
    // are issued ahead of its matrix instructions at two waves per SIMD
#pragma unroll 3
    for (int t = 0; t < kTaps; ++t) {
      const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
      const long long doff = dz * HW + (long long)dy * d.W + dx;
      bool ok[kMT];
      const uint4* src[kMT];
#pragma unroll
      for (int m = 0; m < kMT; ++m) {
        ok[m] = (unsigned)(zz[m] + dz) < (unsigned)d.D && (unsigned)(yy[m] + dy) < (unsigned)d.H &&
                (unsigned)(xx[m] + dx) < (unsigned)d.W;
        src[m] = reinterpret_cast<const uint4*>(X + (ok[m] ? (vv[m] + doff) * kC : 0) + half * 8);
      }
#pragma unroll
      for (int kh = 0; kh < 2; ++kh) {
        const uint4 bw = lw4[((t * kC + row) * kC + kh * 16 + half * 8) / 8];
#pragma unroll
        for (int m = 0; m < kMT; ++m) {
          const uint4 av = ok[m] ? src[m][kh * 2] : make_uint4(0, 0, 0, 0);
          acc[m] = mfma(as_bf8(av), as_bf8(bw), acc[m]);
        }
      }
    }
    // D[i][j]: j = row (output channel), i = 8 (r / 4) + 4 half + r % 4 (voxel in tile)
#pragma unroll
    for (int m = 0; m < kMT; ++m) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const long long v = (tile0 + m) * 32 + 8 * (r / 4) + 4 * half + (r % 4);
        if (v < d.V) {
          float o = acc[m][r] + bj;
          if (RELU) o = fmaxf(o, 0.f);
          if constexpr (OUTF32) static_cast<float*>(Yv)[v * kC + row] = o;
          else static_cast<uint16_t*>(Yv)[v * kC + row] = f2bf(o);
        }
      }
    }
  }
}

// Weight (and bias) gradient partials of one block over voxels
// [blockIdx.x * per, min(V, (blockIdx.x + 1) * per)); per is a multiple of 16.
// part: [gridDim.x][27][32 co][32 ci];  pbias: [gridDim.x][32].
static __global__ void __launch_bounds__(kNB) k_conv3d_wgrad(const uint16_t* __restrict__ X, const uint16_t* __restrict__ G,
                                                      float* __restrict__ part, float* __restrict__ pbias,
                                                      const Dims d, long long per) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row = lane & 31, half = lane >> 5;
  constexpr int kQ = 7;  // taps per wave: t = wv + 4 q
  f32x16 acc[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[q][r] = 0.f;
  float bacc = 0.f;
  const long long HW = (long long)d.H * d.W;
  const long long v_begin = (long long)blockIdx.x * per;
  const long long v_end = min(d.V, v_begin + per);
  for (long long v0 = v_begin; v0 < v_end; v0 += 16) {
    // the 8 voxels of this lane's K group and their coordinates
    const long long vf = v0 + 8 * half;
    int b, z, y, x;
    decompose(vf < d.V ? vf : 0, d, b, z, y, x);
    int cz[8], cy[8], cx[8];
    bool in[8];
    uint16_t ga[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      in[j] = vf + j < v_end;
      cz[j] = z; cy[j] = y; cx[j] = x;
      ga[j] = in[j] ? G[(vf + j) * kC + row] : (uint16_t)0;
      if (++x == d.W) { x = 0; if (++y == d.H) { y = 0; if (++z == d.D) z = 0; } }
    }
    if (wv == 0) {
#pragma unroll
      for (int j = 0; j < 8; ++j) bacc += bf2f(ga[j]);
    }
    const uint4 a4 = make_uint4(ga[0] | ((uint32_t)ga[1] << 16), ga[2] | ((uint32_t)ga[3] << 16),
                                ga[4] | ((uint32_t)ga[5] << 16), ga[6] | ((uint32_t)ga[7] << 16));
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int t = wv + 4 * q;
      if (t < kTaps) {
        const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        const long long doff = dz * HW + (long long)dy * d.W + dx;
        uint16_t xb[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const bool ok = in[j] && (unsigned)(cz[j] + dz) < (unsigned)d.D && (unsigned)(cy[j] + dy) < (unsigned)d.H &&
                          (unsigned)(cx[j] + dx) < (unsigned)d.W;
          xb[j] = ok ? X[(vf + j + doff) * kC + row] : (uint16_t)0;
        }
        const uint4 b4 = make_uint4(xb[0] | ((uint32_t)xb[1] << 16), xb[2] | ((uint32_t)xb[3] << 16),
                                    xb[4] | ((uint32_t)xb[5] << 16), xb[6] | ((uint32_t)xb[7] << 16));
        acc[q] = mfma(as_bf8(a4), as_bf8(b4), acc[q]);
      }
    }
  }
  float* pb = part + (long long)blockIdx.x * kWElems;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int t = wv + 4 * q;
    if (t < kTaps) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int co = 8 * (r / 4) + 4 * half + (r % 4);
        pb[(t * kC + co) * kC + row] = acc[q][r];
      }
    }
  }
  if (wv == 0) {
    bacc += __shfl_xor(bacc, 32, 64);
    if (half == 0) pbias[(long long)blockIdx.x * kC + row] = bacc;
  }
}

// out[i] = sum_p part[p * n + i] (fixed order)
static __global__ void __launch_bounds__(kNB) k_reduce_parts(const float* __restrict__ part, int nparts, int n,
                                                      float* __restrict__ out) {
  const int i = blockIdx.x * kNB + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int p = 0; p < nparts; ++p) s += part[(long long)p * n + i];
  out[i] = s;
}

// ------------------------------------------------------------ elementwise --
// 2x2x2 average pooling: fine dims d (even), coarse dims (d/2)
static __global__ void __launch_bounds__(kNB) k_pool2(const uint16_t* __restrict__ X, uint16_t* __restrict__ Y, const Dims dc) {
  const long long n = dc.V * kC;
  for (long long i = (long long)blockIdx.x * kNB + threadIdx.x; i < n; i += (long long)gridDim.x * kNB) {
    const int c = (int)(i % kC);
    int b, z, y, x;
    decompose(i / kC, dc, b, z, y, x);
    const int W = 2 * dc.W, H = 2 * dc.H, D = 2 * dc.D;
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const long long fv = (((long long)b * D + 2 * z + (k >> 2)) * H + 2 * y + ((k >> 1) & 1)) * W + 2 * x + (k & 1);
      s += bf2f(X[fv * kC + c]);
    }
    Y[i] = f2bf(s * 0.125f);
  }
}

// Y = up2(Xc) + S (S may be null): nearest upsampling of the coarse tensor
static __global__ void __launch_bounds__(kNB) k_up2_add(const uint16_t* __restrict__ Xc, const uint16_t* __restrict__ S,
                                                 uint16_t* __restrict__ Y, const Dims df) {
  const long long n = df.V * kC;
  for (long long i = (long long)blockIdx.x * kNB + threadIdx.x; i < n; i += (long long)gridDim.x * kNB) {
    const int c = (int)(i % kC);
    int b, z, y, x;
    decompose(i / kC, df, b, z, y, x);
    const long long cv = (((long long)b * (df.D / 2) + z / 2) * (df.H / 2) + y / 2) * (df.W / 2) + x / 2;
    float v = bf2f(Xc[cv * kC + c]);
    if (S) v += bf2f(S[i]);
    Y[i] = f2bf(v);
  }
}

// Gc = sum over each 2x2x2 block of Gf (adjoint of up2); coarse dims dc
static __global__ void __launch_bounds__(kNB) k_up2_bwd(const uint16_t* __restrict__ Gf, uint16_t* __restrict__ Gc, const Dims dc) {
  const long long n = dc.V * kC;
  for (long long i = (long long)blockIdx.x * kNB + threadIdx.x; i < n; i += (long long)gridDim.x * kNB) {
    const int c = (int)(i % kC);
    int b, z, y, x;
    decompose(i / kC, dc, b, z, y, x);
    const int W = 2 * dc.W, H = 2 * dc.H, D = 2 * dc.D;
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const long long fv = (((long long)b * D + 2 * z + (k >> 2)) * H + 2 * y + ((k >> 1) & 1)) * W + 2 * x + (k & 1);
      s += bf2f(Gf[fv * kC + c]);
    }
    Gc[i] = f2bf(s);
  }
}

// Gf = Gc / 8 broadcast (adjoint of pool2) + S (may be null); fine dims df
static __global__ void __launch_bounds__(kNB) k_pool2_bwd_add(const uint16_t* __restrict__ Gc, const uint16_t* __restrict__ S,
                                                       uint16_t* __restrict__ Gf, const Dims df) {
  const long long n = df.V * kC;
  for (long long i = (long long)blockIdx.x * kNB + threadIdx.x; i < n; i += (long long)gridDim.x * kNB) {
    const int c = (int)(i % kC);
    int b, z, y, x;
    decompose(i / kC, df, b, z, y, x);
    const long long cv = (((long long)b * (df.D / 2) + z / 2) * (df.H / 2) + y / 2) * (df.W / 2) + x / 2;
    float v = bf2f(Gc[cv * kC + c]) * 0.125f;
    if (S) v += bf2f(S[i]);
    Gf[i] = f2bf(v);
  }
}

// G = G * (Y > 0) (ReLU backward, in place)
static __global__ void __launch_bounds__(kNB) k_relu_mask(uint16_t* __restrict__ G, const uint16_t* __restrict__ Y, long long n) {
  for (long long i = (long long)blockIdx.x * kNB + threadIdx.x; i < n; i += (long long)gridDim.x * kNB)
    if (!(bf2f(Y[i]) > 0.f)) G[i] = 0;
}

// Mean squared error over the first nout channels of Y (FP32) against
// T [V][nout] (bfloat16): G = 2 (Y - T) / cnt (bfloat16, zero for c >= nout),
// FP64 block partials of sum (Y - T)^2.
static __global__ void __launch_bounds__(kNB) k_mse(const float* __restrict__ Y, const uint16_t* __restrict__ T,
                                             uint16_t* __restrict__ G, long long V, int nout, double inv_cnt,
                                             double* __restrict__ partial) {
  __shared__ double red[kNB];
  double acc = 0.0;
  const long long n = V * kC;
  for (long long i = (long long)blockIdx.x * kNB + threadIdx.x; i < n; i += (long long)gridDim.x * kNB) {
    const int c = (int)(i % kC);
    if (c < nout) {
      const double e = (double)Y[i] - (double)bf2f(T[(i / kC) * nout + c]);
      acc += e * e;
      G[i] = f2bf((float)(2.0 * e * inv_cnt));
    } else {
      G[i] = 0;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kNB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Adam (FP32 master weights), step >= 1 via the bias corrections bc1 = 1 - beta1^step, bc2 = 1 - beta2^step.
// omb1 = 1 - beta1 and omb2 = 1 - beta2 come from the host in FP64 (formed in
// FP32, 1 - 0.999f is off by 1.3e-5 relative).
static __global__ void __launch_bounds__(kNB) k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, long long n, float lr, float b1, float omb1,
                                              float b2, float omb2, float eps, float bc1, float bc2) {
  for (long long i = (long long)blockIdx.x * kNB + threadIdx.x; i < n; i += (long long)gridDim.x * kNB) {
    const float gi = g[i];
    const float mi = b1 * m[i] + omb1 * gi;
    const float vi = b2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

// bfloat16 copies of the weights of nconv convolutions stored as FP32
// [nconv][27*32*32 weights + 32 biases]
static __global__ void __launch_bounds__(kNB) k_pack_weights(const float* __restrict__ p, uint16_t* __restrict__ wb, int nconv) {
  const long long n = (long long)nconv * kWElems;
  for (long long i = (long long)blockIdx.x * kNB + threadIdx.x; i < n; i += (long long)gridDim.x * kNB) {
    const long long c = i / kWElems, e = i % kWElems;
    wb[i] = f2bf(p[c * (kWElems + kC) + e]);
  }
}

}  // namespace nn
}  // namespace pn
