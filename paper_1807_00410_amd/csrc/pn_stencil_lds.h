// LDS-tiled stencil apply with one-plane-ahead prefetch (FP32, vacuum
// boundary, padded lattice of pn_kernels.h).
//
// A block owns a TX x TY tile of (x, y) columns and marches a chunk of z
// planes.  Per plane every input coefficient is staged in LDS over the tile
// plus a one-point ring (the x/y neighbours), so the in-plane differences read
// LDS only.  The z differences use a per-thread register window of the
// thread's own column.  All global loads of plane z+1 (own values, the ring,
// the cell parameters) -- and of plane z+2 for the z-face inputs, whose
// z-difference looks one plane up -- are issued right after plane z is staged
// and before plane z's stores.  On CDNA one in-order counter covers loads and
// stores, so a load issued after a store can only be consumed once that store
// has completed; issuing a step ahead and before the stores leaves a whole
// step of compute between every load and its first use, and no wait on the
// stores.
//
// Modes: M_APPLY  y = op(x)                 [NORM: ||y||^2 partials]
//        M_SUPD   s = s - alpha op(x)        [||s||^2 partials]
#pragma once
#include "pn_kernels.h"

namespace pn {

template <int N, int MODE, bool NORM>
__global__ void __launch_bounds__(kBlock) k_stencil_lds(const StencilArgs a) {
  using TB = Table<N>;
  constexpr int NC = TB::NC;
  extern __shared__ float lds[];
  // inside the Krylov loop both launches end once the stop flag is up
  if (a.st != nullptr && (a.st->done || a.st->stop)) return;

  const int ntile = a.ntx * a.nty;
  const int L = xcd_remap(blockIdx.x, a.nblocks);
  const int tb = L % ntile, zc = L / ntile;
  const int tx0 = (tb % a.ntx) * a.TX, ty0 = (tb / a.ntx) * a.TY;
  const int z0 = zc * a.zchunk;
  const int z1 = min(z0 + a.zchunk, a.Ez);
  const int t = threadIdx.x;
  const int TX = a.TX, TY = a.TY, tw = a.TX + 2;
  const int tsz = tw * (a.TY + 2);  // LDS floats per coefficient

  const bool in_tile = t < TX * TY;
  const int lx = in_tile ? t % TX : 0, ly = in_tile ? t / TX : 0;
  const int x = tx0 + lx, y = ty0 + ly;
  const bool act = in_tile && x < a.Ex && y < a.Ey;
  // own column, clamped into the padded lattice for lanes outside it
  const int xc = min(x, a.Ex), yc = min(y, a.Ey);
  const unsigned o = (unsigned)((yc + 1) * a.PX + (xc + 1)) * 4u;
  const int lown = (ly + 1) * tw + (lx + 1);
  // ring slot of this thread: the tile's one-point border
  const int ring = 2 * tw + 2 * TY;
  const bool has_h = t < ring;
  int hi, hj;
  if (t < tw) { hi = t - 1; hj = -1; }
  else if (t < 2 * tw) { hi = t - tw - 1; hj = TY; }
  else { const int r = t - 2 * tw; hj = r >> 1; hi = (r & 1) ? TX : -1; }
  const int hx = min(max(tx0 + hi, -1), a.Ex), hy = min(max(ty0 + hj, -1), a.Ey);
  const unsigned oh = (unsigned)((hy + 1) * a.PX + (hx + 1)) * 4u;
  const int lh = has_h ? (hj + 1) * tw + (hi + 1) : 0;
  // cell parameters: padded cell (x-1, y-1), clamped for lanes outside the lattice
  const unsigned mo = (unsigned)(min(yc, a.ny) * a.CX + min(xc, a.nx)) * 8u;
  const unsigned mcx = (unsigned)a.CX * 8u;
  const bool okx0 = x < a.nx, oky0 = y < a.ny;

  const float* __restrict__ X = static_cast<const float*>(a.x);
  float* __restrict__ Y = static_cast<float*>(a.y);
  const long long cs = a.cs;
  const float tinvh = float(a.tsign * a.invh);
  float alpha = 0.f;
  if constexpr (MODE == M_SUPD) alpha = float(a.st->alpha);

  auto plane = [&](int z) -> long long {  // padded plane offset of lattice plane z, clamped
    z = min(max(z, -1), a.Ez);
    return (long long)__builtin_amdgcn_readfirstlane((z + 1) * a.plane);
  };
  // opaque uniform element offset of (coefficient, plane): see k_stencil
  auto cbase = [&](int k, long long zo) -> long long {
    return (long long)__builtin_amdgcn_readfirstlane((int)((long long)k * cs + zo));
  };
  auto ld = [&](int k, long long zo, unsigned off) -> float { return ldb(X + cbase(k, zo), off); };
  auto cells = [&](int z, float2* c) {
    z = min(max(z, -1), a.nz);
    const float2* __restrict__ mp = a.med32 + (long long)(z + 1) * a.cplane;
    c[0] = ldb(mp, mo); c[1] = ldb(mp, mo + 8u); c[2] = ldb(mp, mo + mcx); c[3] = ldb(mp, mo + mcx + 8u);
  };

  // Register window per input K: z-centred (pz = 0): cur = z, aux = z-1, nxt = z+1
  // (in flight); z-face (pz = 1): cur = z, aux = z+1, nxt = z+2 (in flight).
  float cur[NC], aux[NC], nxt[NC], hc[NC], hn[NC];
  float2 mprev[4], mcur[4], mnext[4];
  {
    const long long p0 = plane(z0), pm = plane(z0 - 1), pp = plane(z0 + 1);
    sfor<NC>([&](auto Kc) {
      constexpr int K = decltype(Kc)::value;
      cur[K] = ld(K, p0, o);
      aux[K] = cls_z(K) ? ld(K, pp, o) : ld(K, pm, o);
      hc[K] = has_h ? ld(K, p0, oh) : 0.f;
    });
    cells(z0 - 1, mprev);
    cells(z0, mcur);
  }

  double nrm0 = 0.0, nrm1 = 0.0;
#pragma clang loop unroll(disable)
  for (int z = z0; z < z1; ++z) {
    // stage plane z
    __syncthreads();
    sfor<NC>([&](auto Kc) {
      constexpr int K = decltype(Kc)::value;
      lds[K * tsz + lown] = cur[K];
      if (has_h) lds[K * tsz + lh] = hc[K];
    });
    __syncthreads();
    // prefetch the next step (before this step's stores)
    {
      const long long p1 = plane(z + 1), p2 = plane(z + 2);
      sfor<NC>([&](auto Kc) {
        constexpr int K = decltype(Kc)::value;
        nxt[K] = ld(K, cls_z(K) ? p2 : p1, o);
        hn[K] = has_h ? ld(K, p1, oh) : 0.f;
      });
      cells(z + 1, mnext);
    }
    // class means of sigma_a and sigma_s (z-major, lower neighbour first)
    float msa[8], mss[8], csa[8], css[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      msa[q] = mprev[q].x; mss[q] = mprev[q].y;
      msa[4 + q] = mcur[q].x; mss[4 + q] = mcur[q].y;
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int px = c & 1, py = (c >> 1) & 1, pz = (c >> 2) & 1;
      float s0 = 0.f, s1 = 0.f;
      int cnt = 0;
#pragma unroll
      for (int dz = 1 - pz; dz < 2; ++dz)
#pragma unroll
        for (int dy = 1 - py; dy < 2; ++dy)
#pragma unroll
          for (int dx = 1 - px; dx < 2; ++dx) {
            s0 += msa[4 * dz + 2 * dy + dx];
            s1 += mss[4 * dz + 2 * dy + dx];
            ++cnt;
          }
      csa[c] = s0 * (1.f / float(cnt));
      css[c] = s1 * (1.f / float(cnt));
    }
    const long long zo = plane(z);
    const bool okz0 = z < a.nz;
    sfor<8>([&](auto Cc) {
      constexpr int c = decltype(Cc)::value;
      if constexpr (TB::class_has_rows(c)) {
        constexpr int ib = TB::class_begin(c);
        constexpr int ie = TB::class_end(c);
        float acc[NC];
        sfor<NC>([&](auto Kc) {
          constexpr int K = decltype(Kc)::value;
          if constexpr (cls_id(K) == c) acc[K] = 0.f;
        });
        float dcur = 0.f;
        sfor<ie - ib>([&](auto Ic) {
          constexpr int I = ib + decltype(Ic)::value;
          constexpr Coupling cp = TB::cpl.v[I];
          constexpr bool first = TB::starts_difference(I);
          if constexpr (first) {
            constexpr int p = cls_axis(cp.kp, cp.d);
            if constexpr (cp.d == 2) {
              dcur = p ? aux[cp.kp] - cur[cp.kp] : cur[cp.kp] - aux[cp.kp];
            } else {
              const int step = (cp.d == 0) ? 1 : tw;
              const float v = lds[cp.kp * tsz + lown + (p ? step : -step)];
              dcur = p ? v - cur[cp.kp] : cur[cp.kp] - v;
            }
          }
          acc[cp.k] = fmadd<float>(float(cp.c), dcur, acc[cp.k]);
        });
        constexpr int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
        const bool ok = act && (cx || okx0) && (cy || oky0) && (cz || okz0);
        if (ok) {
          float cn = 0.f;
          sfor<NC>([&](auto Kc) {
            constexpr int K = decltype(Kc)::value;
            if constexpr (cls_id(K) == c) {
              const long long base = cbase(K, zo);
              const float dg = fmadd<float>(float(a.omg[band_of(K)]), css[c], csa[c]);
              const float out = fmadd<float>(tinvh, acc[K], dg * cur[K]);
              if constexpr (MODE == M_SUPD) {
                const float sn = fmadd<float>(-alpha, out, ldb(Y + base, o));
                stb(Y + base, o, sn);
                cn = fmadd<float>(sn, sn, cn);
              } else {
                stb(Y + base, o, out);
                if constexpr (NORM) cn = fmadd<float>(out, out, cn);
              }
            }
          });
          if constexpr (NORM || MODE == M_SUPD) nrm0 += double(cn);
        }
      }
    });
    // rotate the windows
    sfor<NC>([&](auto Kc) {
      constexpr int K = decltype(Kc)::value;
      if constexpr (cls_z(K) == 1) { cur[K] = aux[K]; aux[K] = nxt[K]; }
      else { aux[K] = cur[K]; cur[K] = nxt[K]; }
      hc[K] = hn[K];
    });
#pragma unroll
    for (int q = 0; q < 4; ++q) { mprev[q] = mcur[q]; mcur[q] = mnext[q]; }
  }

  if constexpr (NORM || MODE == M_SUPD) {
    block_sum2(nrm0, nrm1);
    if (threadIdx.x == 0) {
      a.partials[2 * L] = nrm0;
      a.partials[2 * L + 1] = nrm1;
    }
  }
}

// Allows dynamic LDS above the default limit for the three variants.
template <int N>
hipError_t lds_prepare(size_t shm) {
  const int b = (int)shm;
  hipError_t e = hipFuncSetAttribute((const void*)k_stencil_lds<N, M_SUPD, true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, b);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_stencil_lds<N, M_APPLY, true>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_stencil_lds<N, M_APPLY, false>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, b);
}

// Launch helper: block = TX*TY threads rounded up to a wavefront multiple;
// dynamic LDS = NC * (TX+2) * (TY+2) floats.
template <int N>
hipError_t launch_lds_order(int mode, bool norm, const StencilArgs& a, hipStream_t s) {
  constexpr int NC = (N + 1) * (N + 1);
  const int threads = ((a.TX * a.TY + 63) / 64) * 64;
  const size_t shm = sizeof(float) * (size_t)NC * (a.TX + 2) * (a.TY + 2);
  dim3 grid(a.nblocks), block(threads);
  if (mode == M_SUPD) hipLaunchKernelGGL((k_stencil_lds<N, M_SUPD, true>), grid, block, shm, s, a);
  else if (norm) hipLaunchKernelGGL((k_stencil_lds<N, M_APPLY, true>), grid, block, shm, s, a);
  else hipLaunchKernelGGL((k_stencil_lds<N, M_APPLY, false>), grid, block, shm, s, a);
  return hipGetLastError();
}

}  // namespace pn
