// HIP kernels of the staggered real P_N solver (gfx950).
//
// Stencil apply (matrix-free A x, A^T x).  One thread owns one (x, y) column
// of the staggered lattice and marches a chunk of z planes.  Per input
// coefficient it keeps a two-plane register window in z (the plane above for
// z-face classes, the plane below for z-centred ones), so every vector entry
// is fetched from memory once for its own row and the z-difference; the x/y
// neighbours are re-reads of lines that adjacent lanes / rows already pulled
// into L1/L2.  The RTE parameters (sigma_t, albedo per cell, 8 bytes) are
// averaged on the fly from the 1/2/4/8 cells adjacent to each staggered
// location, with the previous plane of cells kept in registers.
//
// The coupling structure is a compile-time table (pn_tables.h), so the
// per-class bookkeeping, the differences and the coupling weights unroll into
// straight-line FMA code with literal constants.
//
// Krylov bookkeeping: dot products are accumulated in FP64 per thread,
// reduced per wavefront with cross-lane shuffles, per block through LDS in a
// fixed order, and per grid by a one-block finalize kernel that also forms
// the CGLS scalars on the device (no host round trip per iteration).
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

#include "pn_tables.h"

namespace pn {

constexpr int kBlock = 256;
constexpr int kMaxCoeff = 64;

// ------------------------------------------------------------------ state --
struct DevState {
  double gamma;   // ||s||^2 of the current normal-equation residual s = A^T r
  double alpha;   // step length
  double beta;    // direction update factor
  double rr;      // ||r||^2 of the (recursive) residual
  double rr0;     // ||r||^2 at the start of the current inner solve
  double tol2;    // inner stop threshold on rr
  double qq;      // ||A p||^2
  double rtrue2;  // ||Q - A x||^2 from the FP64 residual kernel
  double bb2;     // ||Q||^2
  double nonfinite;
  int iters;      // Krylov iterations so far (all inner solves)
  int max_iters;
  int stop;       // set when the iteration must end after this step's update
  int done;       // set one step later: every kernel returns at once
  int breakdown;
  int pad[3];
};

enum Mode { M_APPLY = 0, M_TRANSR = 1, M_RESID = 2 };

struct StencilArgs {
  int nx, ny, nz;
  int Ex, Ey, Ez;      // thread lattice: n + 1 per axis (vacuum) or n (periodic)
  int periodic;
  int zchunk, nzc, ncb, nblocks;
  double invh;         // 1 / h
  double tsign;        // +1: A, -1: A^T
  double omg[8];       // 1 - g^l, l = 0..7
  int off[kMaxCoeff];  // offset of coefficient k in the vector (elements)
  const float2* med;   // per cell (thresholded sigma_t, albedo)
  const void* x;       // input vector (T); M_TRANSR: r
  const void* x2;      // M_TRANSR: q;  M_RESID: right-hand side (float)
  void* y;             // output vector
  void* y2;            // M_APPLY: optional second copy of y; M_TRANSR: updated r
  DevState* st;        // device scalars (alpha for M_TRANSR, done flag), may be null
  double* partials;    // [nblocks][2] FP64 partial sums, may be null
};

template <class F, int... I>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// Blocks are handed to the 8 XCDs round-robin; give each XCD a contiguous
// range of logical tiles so neighbouring columns / chunks share an L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, slot = b >> 3;
  return (xcd < r) ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c);
template <>
__device__ __forceinline__ float fmadd<float>(float a, float b, float c) { return __fmaf_rn(a, b, c); }
template <>
__device__ __forceinline__ double fmadd<double>(double a, double b, double c) { return __fma_rn(a, b, c); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic block sum of two FP64 values; result valid in thread 0.
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  __shared__ double red[2][kBlock / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) { red[0][w] = a; red[1][w] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int i = 0; i < kBlock / 64; ++i) { s0 += red[0][i]; s1 += red[1][i]; }
    a = s0; b = s1;
  }
}

// --------------------------------------------------------------- stencil --
// T: arithmetic / vector type of the input (float or double).
// TO: output element type.  MODE: M_APPLY  y = op(x)            [+ ||y||^2]
//                                 M_TRANSR r' = r - alpha q, y = A^T r'
//                                          [writes r' to y2; ||y||^2, ||r'||^2]
//                                 M_RESID  y = Q - A x        [||y||^2, ||Q||^2]
template <int N, typename T, int MODE, typename TO>
__global__ void __launch_bounds__(kBlock) k_stencil(const StencilArgs a) {
  using TB = Table<N>;
  constexpr int NC = TB::NC;
  constexpr int NCPL = TB::NCPL;
  // In the Krylov loop the A p launch also ends once the stop flag is up.
  if (a.st != nullptr && (a.st->done || (MODE == M_APPLY && a.st->stop))) return;

  const int L = xcd_remap(blockIdx.x, a.nblocks);
  const int cb = L % a.ncb, zc = L / a.ncb;
  const int col = cb * kBlock + threadIdx.x;
  const bool act = col < a.Ex * a.Ey;
  const int x = act ? col % a.Ex : 0;
  const int y = act ? col / a.Ex : 0;
  const int z0 = zc * a.zchunk;
  const int z1 = min(z0 + a.zchunk, a.Ez);
  const int per = a.periodic;

  const T* __restrict__ X = static_cast<const T*>(a.x);
  const T* __restrict__ X2 = static_cast<const T*>(a.x2);
  const float* __restrict__ RHS = static_cast<const float*>(a.x2);
  TO* __restrict__ Y = static_cast<TO*>(a.y);
  TO* __restrict__ Y2 = static_cast<TO*>(a.y2);
  T alpha = T(0);
  if constexpr (MODE == M_TRANSR) alpha = T(a.st->alpha);
  const T tinvh = T(a.tsign * a.invh);

  double nrm0 = 0.0, nrm1 = 0.0;

  // Flat index of coefficient KP at lattice point (i, j, k); -1 if outside.
  auto index_of = [&](auto KPc, int i, int j, int k) -> int {
    constexpr int KP = decltype(KPc)::value;
    const int ex = a.nx + (per ? 0 : cls_x(KP));
    const int ey = a.ny + (per ? 0 : cls_y(KP));
    const int ez = a.nz + (per ? 0 : cls_z(KP));
    if (per) {
      i = wrapi(i, ex); j = wrapi(j, ey); k = wrapi(k, ez);
    } else if ((unsigned)i >= (unsigned)ex || (unsigned)j >= (unsigned)ey || (unsigned)k >= (unsigned)ez) {
      return -1;
    }
    return a.off[KP] + (k * ey + j) * ex + i;
  };
  auto val = [&](auto KPc, int i, int j, int k) -> T {
    const int idx = index_of(KPc, i, j, k);
    if (idx < 0) return T(0);
    if constexpr (MODE == M_TRANSR) return fmadd<T>(-alpha, X2[idx], X[idx]);
    else return X[idx];
  };
  auto cell = [&](int i, int j, int k) -> float2 {
    if (per) {
      i = wrapi(i, a.nx); j = wrapi(j, a.ny); k = wrapi(k, a.nz);
    } else {
      i = min(max(i, 0), a.nx - 1); j = min(max(j, 0), a.ny - 1); k = min(max(k, 0), a.nz - 1);
    }
    return a.med[(k * a.ny + j) * a.nx + i];
  };

  if (act) {
    T cur[NC], nb[NC];
    sfor<NC>([&](auto KPc) {
      constexpr int KP = decltype(KPc)::value;
      if constexpr (cls_z(KP) == 1) nb[KP] = val(KPc, x, y, z0);
      else cur[KP] = val(KPc, x, y, z0 - 1);
    });
    // cells (x-1|x, y-1|y) of the plane below, index q = 2*dy + dx
    float2 mprev[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) mprev[q] = cell(x - 1 + (q & 1), y - 1 + (q >> 1), z0 - 1);

    for (int z = z0; z < z1; ++z) {
      sfor<NC>([&](auto KPc) {
        constexpr int KP = decltype(KPc)::value;
        if constexpr (cls_z(KP) == 1) { cur[KP] = nb[KP]; nb[KP] = val(KPc, x, y, z + 1); }
        else { nb[KP] = cur[KP]; cur[KP] = val(KPc, x, y, z); }
      });
      float2 mcur[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) mcur[q] = cell(x - 1 + (q & 1), y - 1 + (q >> 1), z);
      // Per-cell sigma_a = sigma_t (1 - albedo) and sigma_s = sigma_t albedo,
      // index c = 4*dz + 2*dy + dx (0 = lower neighbour).  The row diagonal
      // sigma_t - g^l sigma_s is formed as mean(sigma_a) + (1 - g^l) mean(sigma_s):
      // the same number, without the cancellation of sigma_t - sigma_s when the
      // albedo is close to 1.
      T sa[8], ss[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        sa[q] = T(mprev[q].x) * (T(1) - T(mprev[q].y));
        ss[q] = T(mprev[q].x) * T(mprev[q].y);
        sa[4 + q] = T(mcur[q].x) * (T(1) - T(mcur[q].y));
        ss[4 + q] = T(mcur[q].x) * T(mcur[q].y);
      }
      // class means (cells visited z-major, lower neighbour first)
      T csa[8], css[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int px = c & 1, py = (c >> 1) & 1, pz = (c >> 2) & 1;
        T s0 = T(0), s1 = T(0);
        int cnt = 0;
#pragma unroll
        for (int dz = 1 - pz; dz < 2; ++dz)
#pragma unroll
          for (int dy = 1 - py; dy < 2; ++dy)
#pragma unroll
            for (int dx = 1 - px; dx < 2; ++dx) {
              s0 += sa[4 * dz + 2 * dy + dx];
              s1 += ss[4 * dz + 2 * dy + dx];
              ++cnt;
            }
        const T inv = T(1) / T(cnt);
        csa[c] = s0 * inv;
        css[c] = s1 * inv;
      }

      // transport: differences formed once per (input, axis), fanned out to rows
      T acc[NC];
      sfor<NC>([&](auto K) { acc[decltype(K)::value] = T(0); });
      T dcur = T(0);
      sfor<NCPL>([&](auto Ic) {
        constexpr int I = decltype(Ic)::value;
        constexpr Coupling cp = TB::cpl.v[I];
        constexpr bool first = (I == 0) || TB::cpl.v[I - 1].kp != cp.kp || TB::cpl.v[I - 1].d != cp.d;
        if constexpr (first) {
          constexpr int p = cls_axis(cp.kp, cp.d);
          if constexpr (cp.d == 2) {
            dcur = p ? nb[cp.kp] - cur[cp.kp] : cur[cp.kp] - nb[cp.kp];
          } else {
            const int s = p ? 1 : -1;
            const T v = (cp.d == 0) ? val(std::integral_constant<int, cp.kp>{}, x + s, y, z)
                                    : val(std::integral_constant<int, cp.kp>{}, x, y + s, z);
            dcur = p ? v - cur[cp.kp] : cur[cp.kp] - v;
          }
        }
        acc[cp.k] = fmadd<T>(T(cp.c), dcur, acc[cp.k]);
      });

      sfor<NC>([&](auto Kc) {
        constexpr int K = decltype(Kc)::value;
        const int idx = index_of(Kc, x, y, z);
        if (idx >= 0 && (!per || (x < a.nx && y < a.ny))) {
          constexpr int c = cls_id(K);
          const T dg = fmadd<T>(T(a.omg[band_of(K)]), css[c], csa[c]);
          T out = fmadd<T>(tinvh, acc[K], dg * cur[K]);
          if constexpr (MODE == M_RESID) {
            const T q = T(RHS[idx]);
            out = q - out;
            nrm1 += double(q) * double(q);
          }
          Y[idx] = TO(out);
          nrm0 += double(out) * double(out);
          if constexpr (MODE == M_APPLY) {
            if (Y2 != nullptr) Y2[idx] = TO(out);
          }
          if constexpr (MODE == M_TRANSR) {
            Y2[idx] = TO(cur[K]);
            nrm1 += double(cur[K]) * double(cur[K]);
          }
        }
      });
#pragma unroll
      for (int q = 0; q < 4; ++q) mprev[q] = mcur[q];
    }
  }

  if (a.partials != nullptr) {
    block_sum2(nrm0, nrm1);
    if (threadIdx.x == 0) {
      a.partials[2 * L] = nrm0;
      a.partials[2 * L + 1] = nrm1;
    }
  }
}

// ------------------------------------------------------------- finalize --
// Sum of partials[2*i + j] over i < n in a fixed order (one block).
__device__ __forceinline__ void grid_sum2(const double* __restrict__ p, int n, double& s0, double& s1) {
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) { a += p[2 * i]; b += p[2 * i + 1]; }
  __shared__ double red[2][kBlock];
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  s0 = red[0][0];
  s1 = red[1][0];
}

__device__ __forceinline__ bool finite_d(double v) { return v == v && v - v == 0.0; }

// After q = A p:  alpha = gamma / ||q||^2.
__global__ void __launch_bounds__(kBlock) k_fin_alpha(DevState* st, const double* partials, int n) {
  if (st->done) return;
  if (st->stop) {
    if (threadIdx.x == 0) st->done = 1;
    return;
  }
  double qq, unused;
  grid_sum2(partials, n, qq, unused);
  if (threadIdx.x == 0) {
    st->qq = qq;
    if (!(qq > 0.0) || !finite_d(qq)) {
      st->breakdown = 1;
      st->alpha = 0.0;
      st->stop = 1;
      st->done = 1;
    } else {
      st->alpha = st->gamma / qq;
    }
  }
}

// After s = A^T r':  beta = ||s||^2 / gamma, convergence test on ||r'||^2.
__global__ void __launch_bounds__(kBlock) k_fin_beta(DevState* st, const double* partials, int n) {
  if (st->done) return;
  double ss, rr;
  grid_sum2(partials, n, ss, rr);
  if (threadIdx.x == 0) {
    const double g0 = st->gamma;
    st->beta = (g0 > 0.0) ? ss / g0 : 0.0;
    st->gamma = ss;
    st->rr = rr;
    st->iters += 1;
    if (!finite_d(rr) || !finite_d(ss)) { st->breakdown = 1; st->stop = 1; st->nonfinite = 1.0; }
    if (rr <= st->tol2 || st->iters >= st->max_iters || !(ss > 0.0)) st->stop = 1;
  }
}

// After s = A^T r0, p = s:  start of an inner solve.
__global__ void __launch_bounds__(kBlock) k_fin_init(DevState* st, const double* partials, int n, double inner_tol2) {
  double ss, unused;
  grid_sum2(partials, n, ss, unused);
  if (threadIdx.x == 0) {
    st->gamma = ss;
    st->rr0 = st->rr;
    st->tol2 = inner_tol2 * st->rr;
    st->stop = (ss > 0.0 && finite_d(ss)) ? 0 : 1;
    st->done = 0;
    st->breakdown = 0;
    st->alpha = 0.0;
    st->beta = 0.0;
  }
}

// After r = Q - A x (FP64):  true residual and ||Q||^2.
__global__ void __launch_bounds__(kBlock) k_fin_resid(DevState* st, const double* partials, int n) {
  double rr, bb;
  grid_sum2(partials, n, rr, bb);
  if (threadIdx.x == 0) {
    st->rtrue2 = rr;
    st->bb2 = bb;
    st->rr = rr;
  }
}

// ---------------------------------------------------------------- vector --
// x += alpha p;  p = s + beta p
template <typename T>
__global__ void __launch_bounds__(kBlock) k_update_xp(T* __restrict__ x, T* __restrict__ p,
                                                      const T* __restrict__ s, long n, const DevState* st) {
  if (st->done) return;
  const T al = T(st->alpha), be = T(st->beta);
  const long stride = (long)gridDim.x * kBlock;
  if constexpr (sizeof(T) == 4) {
    const long n4 = n >> 2;
    float4* x4 = reinterpret_cast<float4*>(x);
    float4* p4 = reinterpret_cast<float4*>(p);
    const float4* s4 = reinterpret_cast<const float4*>(s);
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride) {
      float4 pv = p4[i], xv = x4[i], sv = s4[i];
      xv.x = __fmaf_rn(al, pv.x, xv.x); xv.y = __fmaf_rn(al, pv.y, xv.y);
      xv.z = __fmaf_rn(al, pv.z, xv.z); xv.w = __fmaf_rn(al, pv.w, xv.w);
      pv.x = __fmaf_rn(be, pv.x, sv.x); pv.y = __fmaf_rn(be, pv.y, sv.y);
      pv.z = __fmaf_rn(be, pv.z, sv.z); pv.w = __fmaf_rn(be, pv.w, sv.w);
      x4[i] = xv;
      p4[i] = pv;
    }
    for (long i = (n4 << 2) + (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
      const T pv = p[i];
      x[i] = fmadd<T>(al, pv, x[i]);
      p[i] = fmadd<T>(be, pv, s[i]);
    }
  } else {
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
      const T pv = p[i];
      x[i] = fmadd<T>(al, pv, x[i]);
      p[i] = fmadd<T>(be, pv, s[i]);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T* __restrict__ v, long n, T value) {
  const long stride = (long)gridDim.x * kBlock;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) v[i] = value;
}

// x64 += d (refinement update)
template <typename TD>
__global__ void __launch_bounds__(kBlock) k_add_to64(double* __restrict__ x, const TD* __restrict__ d, long n) {
  const long stride = (long)gridDim.x * kBlock;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) x[i] += double(d[i]);
}

// Thresholds sigma_t, packs (sigma_t, albedo) per cell, flags NaN / Inf.
__global__ void __launch_bounds__(kBlock) k_medium_prep(const float* __restrict__ sigma_t,
                                                        const float* __restrict__ albedo, float thr,
                                                        float2* __restrict__ out, long n, int* bad) {
  const long stride = (long)gridDim.x * kBlock;
  int b = 0;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const float s = sigma_t[i], al = albedo[i];
    if (!isfinite(s) || !isfinite(al)) b = 1;
    out[i] = make_float2(fmaxf(s, thr), al);
  }
  if (b) atomicOr(bad, 1);
}

// Flags NaN / Inf in a float vector.
__global__ void __launch_bounds__(kBlock) k_check_finite(const float* __restrict__ v, long n, int* bad) {
  const long stride = (long)gridDim.x * kBlock;
  int b = 0;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
    if (!isfinite(v[i])) b = 1;
  if (b) atomicOr(bad, 1);
}

}  // namespace pn
