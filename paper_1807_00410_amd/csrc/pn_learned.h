// Kernels that connect the solver's padded lattice with the network's
// channels-last cell tensors (learned initial guess and correction).
//
// Network grid: the cell grid rounded up to multiples of 8 (nx8 x ny8 x nz8),
// cells beyond the medium holding zeros.  Input channels per cell:
//   0: sigma_t h (thresholded), 1: sigma_a h = sigma_t (1 - albedo) h,
//   2 + k (k < 16): coefficient k of the source (a lattice vector: the
//      emission Q, or a residual) at the lattice point with the cell's
//      indices, divided by the largest |value| of these over all cells;
//   the rest zero.  An isotropic emission fills channel 2 only.
// Output / target channel k < 16 holds coefficient k (bands l <= 3) at the
// lattice point with the cell's indices (the cell centre for class (0,0,0),
// its lower faces / edges / corner otherwise); the far-boundary points of
// face-centred classes are not represented (set to zero).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pn_kernels.h"
#include "pn_nn_kernels.h"

namespace pn {

constexpr int kNetOut = 16;  // coefficients predicted by the network (P3)

// Where coefficient k of a lattice vector keeps the point with cell indices
// (x, y, z): base[k] + z * sz[k] + y * sy[k] + x (padded or packed layout).
struct NetGeom {
  int nx, ny, nz;      // cells
  int nx8, ny8, nz8;   // network grid
  int CX, CY;          // padded cell pitches (cells nx + 2, ny + 2)
  int nk;              // min(kNetOut, number of coefficients)
  double h;
  long long base[kNetOut];
  long long sz[kNetOut];
  int sy[kNetOut];
};

__device__ __forceinline__ long long lat(const NetGeom& g, int k, int x, int y, int z) {
  return g.base[k] + (long long)z * g.sz[k] + (long long)y * g.sy[k] + x;
}

// max |v| over the cells and the coefficients k < nk of an FP32 lattice vector
// (float bits combined with atomicMax, valid for non-negative floats; *out
// zeroed first).
static __global__ void __launch_bounds__(kBlock) k_src_absmax(const float* __restrict__ v, const NetGeom g,
                                                              unsigned* __restrict__ out) {
  float m = 0.f;
  const long long n = (long long)g.nx * g.ny * g.nz * g.nk;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
    const int k = (int)(i % g.nk);
    const long long c = i / g.nk;
    const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / ((long long)g.nx * g.ny));
    m = fmaxf(m, fabsf(v[lat(g, k, x, y, z)]));
  }
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// Network input of the medium (padded cells (sigma_t, albedo)) and the source.
static __global__ void __launch_bounds__(kBlock) k_net_features(const float2* __restrict__ med,
                                                                const float* __restrict__ src, const NetGeom g,
                                                                const unsigned* __restrict__ absmax,
                                                                uint16_t* __restrict__ x) {
  const float mx = __uint_as_float(*absmax);
  const float inv = mx > 0.f ? 1.f / mx : 0.f;
  const float h = (float)g.h;
  const long long n = (long long)g.nx8 * g.ny8 * g.nz8;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
    const int cx = (int)(i % g.nx8), cy = (int)((i / g.nx8) % g.ny8), cz = (int)(i / ((long long)g.nx8 * g.ny8));
    uint16_t f[nn::kC];
#pragma unroll
    for (int c = 0; c < nn::kC; ++c) f[c] = 0;
    if (cx < g.nx && cy < g.ny && cz < g.nz) {
      const float2 m = med[((long long)(cz + 1) * g.CY + (cy + 1)) * g.CX + (cx + 1)];
      f[0] = nn::f2bf(m.x * h);
      f[1] = nn::f2bf(m.x * (1.f - m.y) * h);
#pragma unroll
      for (int k = 0; k < kNetOut; ++k)
        if (k < g.nk) f[2 + k] = nn::f2bf(src[lat(g, k, cx, cy, cz)] * inv);
    }
    uint4* o = reinterpret_cast<uint4*>(x + i * nn::kC);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      o[q] = make_uint4(f[8 * q] | ((uint32_t)f[8 * q + 1] << 16), f[8 * q + 2] | ((uint32_t)f[8 * q + 3] << 16),
                        f[8 * q + 4] | ((uint32_t)f[8 * q + 5] << 16), f[8 * q + 6] | ((uint32_t)f[8 * q + 7] << 16));
  }
}

// u (FP64 lattice, zero on entry) <- network output y [cells8][32] for
// coefficients k < nk at the lattice points with cell indices.
static __global__ void __launch_bounds__(kBlock) k_net_to_lattice(const float* __restrict__ y, const NetGeom g,
                                                                  double* __restrict__ u) {
  const long long n = (long long)g.nx * g.ny * g.nz * g.nk;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
    const int k = (int)(i % g.nk);
    const long long c = i / g.nk;
    const int x = (int)(c % g.nx), yy = (int)((c / g.nx) % g.ny), z = (int)(c / ((long long)g.nx * g.ny));
    const long long cell8 = ((long long)z * g.ny8 + yy) * g.nx8 + x;
    u[lat(g, k, x, yy, z)] = (double)y[cell8 * nn::kC + k];
  }
}

// max |coefficient 0| of an FP64 lattice vector over the cells (FP64 block
// partial maxima).
// (u - sub when sub != NULL)
static __global__ void __launch_bounds__(kBlock) k_coef0_absmax(const double* __restrict__ u,
                                                                const double* __restrict__ sub, const NetGeom g,
                                                                double* __restrict__ partial) {
  __shared__ double red[kBlock];
  double s = 0.0;
  const long long n = (long long)g.nx * g.ny * g.nz;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
    const int x = (int)(i % g.nx), y = (int)((i / g.nx) % g.ny), z = (int)(i / ((long long)g.nx * g.ny));
    const long long j = lat(g, 0, x, y, z);
    s = fmax(s, fabs(u[j] - (sub != nullptr ? sub[j] : 0.0)));
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Training target [cells8][kNetOut] (bfloat16) from an FP64 lattice
// solution u (minus sub when sub != NULL: a remaining correction), divided by
// max |coefficient 0| (block maxima in `partial`).
static __global__ void __launch_bounds__(kBlock) k_net_targets(const double* __restrict__ u,
                                                               const double* __restrict__ sub, const NetGeom g,
                                                               const double* __restrict__ partial, int nparts,
                                                               uint16_t* __restrict__ t) {
  double mx = 0.0;
  for (int p = 0; p < nparts; ++p) mx = fmax(mx, partial[p]);
  const double sc = mx > 0.0 ? 1.0 / mx : 0.0;
  const long long n = (long long)g.nx8 * g.ny8 * g.nz8 * kNetOut;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
    const int k = (int)(i % kNetOut);
    const long long c = i / kNetOut;
    const int x = (int)(c % g.nx8), y = (int)((c / g.nx8) % g.ny8), z = (int)(c / ((long long)g.nx8 * g.ny8));
    float v = 0.f;
    if (k < g.nk && x < g.nx && y < g.ny && z < g.nz)
      v = (float)((u[lat(g, k, x, y, z)] - (sub != nullptr ? sub[lat(g, k, x, y, z)] : 0.0)) * sc);
    t[i] = nn::f2bf(v);
  }
}

// x = a x + s u (FP64)
static __global__ void __launch_bounds__(kBlock) k_axpby64(double* __restrict__ x, const double* __restrict__ u,
                                                           double a, double s, long n) {
  const long stride = (long)gridDim.x * kBlock;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) x[i] = a * x[i] + s * u[i];
}

}  // namespace pn
