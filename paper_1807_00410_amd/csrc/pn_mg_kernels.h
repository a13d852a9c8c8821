// Kernels of the multigrid preconditioner (structures and design notes in
// pn_mg.h).
#pragma once
#include <hip/hip_runtime.h>

#include "pn_kernels.h"
#include "pn_mg.h"

namespace pn {

// A level holds at most a few million points per slot: 32-bit local indices.
__device__ __forceinline__ long long mg_at(const MgGeom& g, int s, int x, int y, int z) {
  return g.off[s] + (long long)((z * g.ext[s][1] + y) * g.ext[s][0] + x);
}

__device__ __forceinline__ void mg_xyz(const MgGeom& g, int s, int i, int& x, int& y, int& z) {
  const unsigned ex = (unsigned)g.ext[s][0], ey = (unsigned)g.ext[s][1];
  const unsigned t = (unsigned)i / ex;
  x = i - (int)(t * ex);
  z = (int)(t / ey);
  y = (int)t - z * (int)ey;
}

__device__ __forceinline__ int mg_points(const MgGeom& g, int s) { return g.ext[s][0] * g.ext[s][1] * g.ext[s][2]; }

// Every Jacobi step uses this reciprocal of the diagonal (the same fixed
// scaling in every sweep, so the V-cycle stays symmetric).
__device__ __forceinline__ float mg_rcp(float d) { return __builtin_amdgcn_rcpf(d); }

// Fine face weight of slot s between the padded point pidx and pidx + e_d.
__device__ __forceinline__ double mg_fine_w(const MgFine& f, const MgTerms* __restrict__ t,
                                            const float* __restrict__ invdo, int s, long long pidx, int d) {
  const long long stride = d == 0 ? 1 : (d == 1 ? (long long)f.PX : (long long)f.PX * f.PY);
  const long long q = pidx + (1 - f.cls[s][d]) * stride;  // the odd point between the two
  double w = 0.0;
  for (int i = 0; i < t->n[s][d]; ++i) w += (double)t->c2[s][d][i] * (double)invdo[(long long)t->j[s][d][i] * f.cs + q];
  return w;
}

// Level-1 operator {diag, w_x, w_y, w_z} (w_d: weight to the + neighbour):
// sums over the aggregate's children of the fine operator, internal faces
// cancelling.  m32: 1 / diag(S) in the even slots; invdo: 1 / d_o in the odd
// slots.  Grid: (blocks, slots).
static __global__ void __launch_bounds__(kBlock) k_mg_setup1(const MgFine f, const MgGeom g1,
                                                             const MgTerms* __restrict__ t,
                                                             const float* __restrict__ m32,
                                                             const float* __restrict__ invdo, double invh2,
                                                             float4* __restrict__ op, float* __restrict__ idg) {
  const int s = blockIdx.y;
  const int n = mg_points(g1, s);
  const int fe[3] = {f.ext[s][0], f.ext[s][1], f.ext[s][2]};
  const long long stride[3] = {1, (long long)f.PX, (long long)f.PX * f.PY};
  const long long base = (long long)f.k[s] * f.cs;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    int X[3];
    mg_xyz(g1, s, i, X[0], X[1], X[2]);
    double diag = 0.0, wp[3] = {0.0, 0.0, 0.0}, wm[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < 8; ++c) {
      const int cc[3] = {c & 1, (c >> 1) & 1, c >> 2};
      const int xc[3] = {2 * X[0] + cc[0], 2 * X[1] + cc[1], 2 * X[2] + cc[2]};
      if (xc[0] >= fe[0] || xc[1] >= fe[1] || xc[2] >= fe[2]) continue;
      const long long pidx = ((long long)(xc[2] + 1) * f.PY + (xc[1] + 1)) * f.PX + (xc[0] + 1);
      double all = 0.0, kept = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double wpl = invh2 * mg_fine_w(f, t, invdo, s, pidx, d);
        const double wmi = invh2 * mg_fine_w(f, t, invdo, s, pidx - stride[d], d);
        all += wpl + wmi;
        const bool has_p = xc[d] + 1 < fe[d];
        if (!(cc[d] == 0 && has_p)) kept += wpl;  // + face not internal
        if (cc[d] == 0) kept += wmi;              // - face not internal (cc = 1: the sibling 2X)
        if (cc[d] == 1 && has_p) wp[d] += wpl;
        if (cc[d] == 0 && xc[d] >= 1) wm[d] += wmi;
      }
      const double de = 1.0 / (double)m32[base + pidx] - all;  // d_e(x)
      diag += fmax(de, 0.0) + kept;
    }
    const double off = wp[0] + wp[1] + wp[2] + wm[0] + wm[1] + wm[2];
    diag = fmax(diag, (1.0 + 1e-6) * off);
    op[g1.off[s] + i] = make_float4((float)diag, (float)wp[0], (float)wp[1], (float)wp[2]);
    idg[g1.off[s] + i] = mg_rcp((float)diag);
  }
}

// Galerkin coarsening of an explicit level (aggregates of 2 x 2 x 2).
static __global__ void __launch_bounds__(kBlock) k_mg_coarsen(const MgGeom gf, const MgGeom gc,
                                                              const float4* __restrict__ opf,
                                                              float4* __restrict__ opc, float* __restrict__ idgc) {
  const int s = blockIdx.y;
  const int n = mg_points(gc, s);
  const int fe[3] = {gf.ext[s][0], gf.ext[s][1], gf.ext[s][2]};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    int X[3];
    mg_xyz(gc, s, i, X[0], X[1], X[2]);
    double diag = 0.0, wp[3] = {0.0, 0.0, 0.0}, wm[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < 8; ++c) {
      const int cc[3] = {c & 1, (c >> 1) & 1, c >> 2};
      const int xc[3] = {2 * X[0] + cc[0], 2 * X[1] + cc[1], 2 * X[2] + cc[2]};
      if (xc[0] >= fe[0] || xc[1] >= fe[1] || xc[2] >= fe[2]) continue;
      const float4 o = opf[mg_at(gf, s, xc[0], xc[1], xc[2])];
      const double w[3] = {o.y, o.z, o.w};
      diag += (double)o.x;
      for (int d = 0; d < 3; ++d) {
        const bool has_p = xc[d] + 1 < fe[d];
        if (cc[d] == 0 && has_p) diag -= 2.0 * w[d];  // internal pair
        if (cc[d] == 1 && has_p) wp[d] += w[d];
        if (cc[d] == 0 && xc[d] >= 1) {
          int xm[3] = {xc[0], xc[1], xc[2]};
          xm[d] -= 1;
          const float4 om = opf[mg_at(gf, s, xm[0], xm[1], xm[2])];
          wm[d] += d == 0 ? (double)om.y : (d == 1 ? (double)om.z : (double)om.w);
        }
      }
    }
    const double off = wp[0] + wp[1] + wp[2] + wm[0] + wm[1] + wm[2];
    diag = fmax(diag, (1.0 + 1e-6) * off);
    opc[gc.off[s] + i] = make_float4((float)diag, (float)wp[0], (float)wp[1], (float)wp[2]);
    idgc[gc.off[s] + i] = mg_rcp((float)diag);
  }
}

// r1 = P^T r: the fine residual (even slots of the padded r) summed over each
// aggregate, and z1 = omega r1 / diag (the first damped Jacobi sweep of the
// level-1 V-cycle, from zero).  One thread per aggregate: a wave reads 128
// consecutive fine x of each of its four (y, z) rows (tiles of 16 x 16 fine
// columns read this layout in 64-byte pieces and were measured 2x slower).
static __global__ void __launch_bounds__(kBlock) k_mg_restrict0(const MgFine f, const MgGeom g1,
                                                                const float* __restrict__ r,
                                                                const float* __restrict__ idg1,
                                                                float* __restrict__ r1, float* __restrict__ z1,
                                                                float omega, const DevState* __restrict__ st) {
  if (st->stop) return;
  const int s = blockIdx.y;
  const int n = mg_points(g1, s);
  const int fe[3] = {f.ext[s][0], f.ext[s][1], f.ext[s][2]};
  const float* rs = r + (long long)f.k[s] * f.cs;
  const int PX = f.PX, PY = f.PY;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    int X, Y, Z;
    mg_xyz(g1, s, i, X, Y, Z);
    float acc = 0.f;
    for (int c = 0; c < 8; ++c) {
      const int x = 2 * X + (c & 1), y = 2 * Y + ((c >> 1) & 1), z = 2 * Z + (c >> 2);
      if (x >= fe[0] || y >= fe[1] || z >= fe[2]) continue;
      acc += rs[((z + 1) * PY + (y + 1)) * PX + (x + 1)];
    }
    const long long j = g1.off[s] + i;
    r1[j] = acc;
    z1[j] = omega * acc * idg1[j];
  }
}

// (A z)(x) - diag(x) z(x) for the explicit operator, z given pointwise by ZF.
template <typename ZF>
__device__ __forceinline__ float mg_offdiag(const MgGeom& g, int s, const float4* __restrict__ op, const float4& o,
                                            int x, int y, int z, ZF zf) {
  const int e[3] = {g.ext[s][0], g.ext[s][1], g.ext[s][2]};
  float acc = 0.f;
  if (x + 1 < e[0]) acc -= o.y * zf(x + 1, y, z);
  if (y + 1 < e[1]) acc -= o.z * zf(x, y + 1, z);
  if (z + 1 < e[2]) acc -= o.w * zf(x, y, z + 1);
  if (x >= 1) acc -= op[mg_at(g, s, x - 1, y, z)].y * zf(x - 1, y, z);
  if (y >= 1) acc -= op[mg_at(g, s, x, y - 1, z)].z * zf(x, y - 1, z);
  if (z >= 1) acc -= op[mg_at(g, s, x, y, z - 1)].w * zf(x, y, z - 1);
  return acc;
}

// Tiles of the aggregating down pass: 16 x 16 points (x, y) per block of 256
// threads, each thread two z planes (one coarse plane); a wave holds four
// rows of 16, so the x partner of a lane is lane ^ 1 and the y partner
// lane ^ 16, and the 2 x 2 x 2 sums close with two shuffles.  Grid: (tiles of
// the (x, y) extent, coarse z planes, slots).
constexpr int kMgTile = 16;

__device__ __forceinline__ float mg_quad_sum(float v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, kMgTile);
  return v;
}

// Down the V-cycle at level L (z_L = omega r_L / diag already formed):
// r_{L+1} = P^T (r_L - A_L z_L) and the first sweep of level L + 1, z_{L+1} =
// omega r_{L+1} / diag.  Tiled over the points of level L (above).
static __global__ void __launch_bounds__(kBlock) k_mg_down(const MgGeom gf, const MgGeom gc,
                                                           const float4* __restrict__ op, const float* __restrict__ r,
                                                           const float* __restrict__ zl,
                                                           const float* __restrict__ idgc, float* __restrict__ rc,
                                                           float* __restrict__ zc, float omega,
                                                           const DevState* __restrict__ st) {
  if (st->stop) return;
  const int s = blockIdx.z, Z = blockIdx.y;
  const int fx = gf.ext[s][0], fy = gf.ext[s][1], fz = gf.ext[s][2];
  const int ntx = (fx + kMgTile - 1) / kMgTile;
  const int x = (blockIdx.x % ntx) * kMgTile + (threadIdx.x & (kMgTile - 1));
  const int y = (blockIdx.x / ntx) * kMgTile + (threadIdx.x / kMgTile);
  auto zf = [&](int xx, int yy, int zz) { return zl[mg_at(gf, s, xx, yy, zz)]; };
  float acc = 0.f;
  if (x < fx && y < fy) {
    for (int z = 2 * Z; z < 2 * Z + 2 && z < fz; ++z) {
      const long long j = mg_at(gf, s, x, y, z);
      const float4 o = op[j];
      acc += r[j] - (o.x * zl[j] + mg_offdiag(gf, s, op, o, x, y, z, zf));
    }
  }
  acc = mg_quad_sum(acc);
  const int X = x >> 1, Y = y >> 1;
  if (!(x & 1) && !(y & 1) && X < gc.ext[s][0] && Y < gc.ext[s][1] && Z < gc.ext[s][2]) {
    const long long jc = mg_at(gc, s, X, Y, Z);
    rc[jc] = acc;
    zc[jc] = omega * acc * idgc[jc];
  }
}

// Up the V-cycle at level L: z' = z_L + P z_{L+1}, then one damped Jacobi
// sweep z'' = z' + omega (r_L - A_L z') / diag into zo.  With `partials`,
// also the block sums of <r_L, z''> (level 1: the coarse part of <r, B r>).
static __global__ void __launch_bounds__(kBlock) k_mg_up(const MgGeom gf, const MgGeom gc,
                                                         const float4* __restrict__ op, const float* __restrict__ r,
                                                         const float* __restrict__ zl, const float* __restrict__ zc,
                                                         float* __restrict__ zo, float omega,
                                                         double* __restrict__ partials,
                                                         const DevState* __restrict__ st) {
  if (st->stop) return;
  const int s = blockIdx.y;
  const int n = mg_points(gf, s);
  auto zf = [&](int x, int y, int z) {
    return zl[mg_at(gf, s, x, y, z)] + zc[mg_at(gc, s, x >> 1, y >> 1, z >> 1)];
  };
  double s0 = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    int x, y, z;
    mg_xyz(gf, s, i, x, y, z);
    const long long j = gf.off[s] + i;
    const float4 o = op[j];
    const float zp = zf(x, y, z);
    const float rv = r[j];
    const float out = zp + omega * (rv - (o.x * zp + mg_offdiag(gf, s, op, o, x, y, z, zf))) * mg_rcp(o.x);
    zo[j] = out;
    s0 += (double)(rv * out);
  }
  if (partials) {
    double unused = 0.0;
    block_sum2(s0, unused);
    if (threadIdx.x == 0) {
      const int b = blockIdx.y * gridDim.x + blockIdx.x;
      partials[2 * b] = s0;
      partials[2 * b + 1] = 0.0;
    }
  }
}

// Coarsest level (at most kMgCoarseMax points, one block): `sweeps` damped
// Jacobi sweeps from zero in LDS -- the first one, omega r / diag, formed by
// the kernel before (in z) -- each thread keeping the neighbour indices and
// weights of its points in registers; the result in z.  With `partials`,
// partials[0] = <r, z> (the coarsest level is level 1).
constexpr int kMgCoarseMax = 2048;
constexpr int kMgCoarsePer = kMgCoarseMax / kFinBlock;

static __global__ void __launch_bounds__(kFinBlock) k_mg_coarsest(const MgGeom g, const float4* __restrict__ op,
                                                                  const float* __restrict__ r, float* __restrict__ z,
                                                                  int sweeps, float omega,
                                                                  double* __restrict__ partials,
                                                                  const DevState* __restrict__ st) {
  __shared__ float za[kMgCoarseMax], zb[kMgCoarseMax];
  __shared__ double red[kFinBlock / 64];
  if (st->stop) return;
  const int n = (int)g.off[g.nk];
  int nb[kMgCoarsePer][6];
  float w[kMgCoarsePer][6], dg[kMgCoarsePer], idg[kMgCoarsePer], rv[kMgCoarsePer];
  for (int t = 0; t < kMgCoarsePer; ++t) {
    const int i = threadIdx.x + t * kFinBlock;
    dg[t] = 1.f; idg[t] = 0.f; rv[t] = 0.f;
    for (int e = 0; e < 6; ++e) { nb[t][e] = i; w[t][e] = 0.f; }
    if (i >= n) continue;
    int s = 0;
    while (s + 1 < g.nk && i >= (int)g.off[s + 1]) ++s;
    int x, y, zz;
    mg_xyz(g, s, i - (int)g.off[s], x, y, zz);
    const int e3[3] = {g.ext[s][0], g.ext[s][1], g.ext[s][2]};
    const int c3[3] = {x, y, zz};
    const float4 o = op[i];
    const float wp[3] = {o.y, o.z, o.w};
    dg[t] = o.x;
    idg[t] = mg_rcp(o.x);
    rv[t] = r[i];
    for (int d = 0; d < 3; ++d) {
      const int stride = d == 0 ? 1 : (d == 1 ? e3[0] : e3[0] * e3[1]);
      if (c3[d] + 1 < e3[d]) { nb[t][2 * d] = i + stride; w[t][2 * d] = wp[d]; }
      if (c3[d] >= 1) {
        const float4 om = op[i - stride];
        nb[t][2 * d + 1] = i - stride;
        w[t][2 * d + 1] = d == 0 ? om.y : (d == 1 ? om.z : om.w);
      }
    }
    za[i] = z[i];
  }
  __syncthreads();
  float* cur = za;
  float* nxt = zb;
  for (int sw = 1; sw < sweeps; ++sw) {
    for (int t = 0; t < kMgCoarsePer; ++t) {
      const int i = threadIdx.x + t * kFinBlock;
      if (i >= n) continue;
      float az = dg[t] * cur[i];
      for (int e = 0; e < 6; ++e) az -= w[t][e] * cur[nb[t][e]];
      nxt[i] = cur[i] + omega * (rv[t] - az) * idg[t];
    }
    __syncthreads();
    float* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  double s0 = 0.0;
  for (int t = 0; t < kMgCoarsePer; ++t) {
    const int i = threadIdx.x + t * kFinBlock;
    if (i >= n) continue;
    z[i] = cur[i];
    s0 += (double)(rv[t] * cur[i]);
  }
  if (partials) {
    s0 = wave_sum(s0);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s0;
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0.0;
      for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) a += red[wv];
      partials[0] = a;
      partials[1] = 0.0;
    }
  }
}

// After the r update: <r, M r> kept for the coarse part, <r, r> tested.
// INIT: the start of an inner solve (as fin_init_pcg, gamma formed later).
template <bool INIT>
__global__ void __launch_bounds__(kFinBlock) k_fin_rz_mg(DevState* st, const double* partials, int n,
                                                         double inner_tol2) {
  if (!INIT && (st->done || st->stop)) return;
  double rz, rr;
  grid_sum2(partials, n, rz, rr);
  if (threadIdx.x == 0) {
    st->rzf = rz;
    st->rr = rr;
    if (INIT) {
      st->rr0 = st->rtrue2;
      st->tol2 = inner_tol2 * st->rtrue2;
      st->stop = (rz > 0.0 && finite_d(rz) && rr > st->tol2) ? 0 : 1;
      st->done = 0;
      st->breakdown = 0;
      st->alpha = 0.0;
      st->beta = 0.0;
      st->gamma = 0.0;
    } else {
      st->iters += 1;
      if (!finite_d(rr) || !finite_d(rz)) { st->breakdown = 1; st->stop = 1; st->nonfinite = 1.0; }
      if (rr <= st->tol2 || st->iters >= st->max_iters || !(rz > 0.0)) st->stop = 1;
    }
  }
}

// One iteration's scalars after the V-cycle: <r, M r> and <r, r> from the
// even-row pass's partials (pr, nr pairs), <P^T r, V(P^T r)> from the
// V-cycle's (pc, nc); the stop test on <r, r>, then gamma' = <r, B r> =
// omega_f <r, M r> + <P^T r, V(P^T r)> and beta = gamma' / gamma.  (The
// V-cycle of the last iteration runs before its stop test: one V-cycle more
// per inner solve, one kernel less per iteration.)
__global__ void __launch_bounds__(kFinBlock) k_fin_iter_mg(DevState* st, const double* pr, int nr,
                                                           const double* pc, int nc, double omega_f) {
  if (st->done || st->stop) return;
  double rz, rr, cz, unused;
  grid_sum2(pr, nr, rz, rr);
  grid_sum2(pc, nc, cz, unused);
  if (threadIdx.x == 0) {
    st->rzf = rz;
    st->rr = rr;
    st->iters += 1;
    if (!finite_d(rr) || !finite_d(rz)) { st->breakdown = 1; st->stop = 1; st->nonfinite = 1.0; }
    if (rr <= st->tol2 || st->iters >= st->max_iters || !(rz > 0.0)) st->stop = 1;
    const double gnew = omega_f * rz + cz;
    if (!st->stop) {
      if (!(gnew > 0.0) || !finite_d(gnew)) {
        st->breakdown = 1;
        st->stop = 1;
        st->beta = 0.0;
      } else {
        st->beta = gnew / st->gamma;
        st->gamma = gnew;
      }
    }
  }
}

// gamma' = <r, B r> = omega_f <r, M r> + <P^T r, V(P^T r)>, beta = gamma' / gamma.
template <bool INIT>
__global__ void __launch_bounds__(kFinBlock) k_fin_beta_mg(DevState* st, const double* partials, int n,
                                                           double omega_f) {
  if (st->done || st->stop) return;
  double cz, unused;
  grid_sum2(partials, n, cz, unused);
  if (threadIdx.x == 0) {
    const double gnew = omega_f * st->rzf + cz;
    if (!(gnew > 0.0) || !finite_d(gnew)) {
      st->breakdown = 1;
      st->stop = 1;
      st->beta = 0.0;
    } else {
      st->beta = INIT ? 0.0 : gnew / st->gamma;
      st->gamma = gnew;
    }
  }
}

// OP 2: x += alpha p, p = B r + beta p;  OP 4 (start): p = B r, with
// B r = omega_f m r + z1 at the point's aggregate (zero outside the class
// extent, where r and p stay zero).
template <int OP>
__global__ void __launch_bounds__(kBlock) k_pcg_vec_mg(float* __restrict__ x, const float* __restrict__ r,
                                                       float* __restrict__ p, const uint16_t* __restrict__ m,
                                                       const MgFine f, const MgGeom g1, const float* __restrict__ z1,
                                                       float omega_f, const DevState* __restrict__ st) {
  if (OP == 2 && st->done) return;
  const int s = blockIdx.y;
  const long long base = (long long)f.k[s] * f.cs;
  const long long n4 = f.cs >> 2;
  const long long stride = (long long)gridDim.x * kBlock;
  const float al = OP == 2 ? float(st->alpha) : 0.f, be = OP == 2 ? float(st->beta) : 0.f;
  const int fx = f.ext[s][0], fy = f.ext[s][1], fz = f.ext[s][2];
  const int ex1 = g1.ext[s][0], ey1 = g1.ext[s][1];
  const float* zs = z1 + g1.off[s];
  float4* x4 = reinterpret_cast<float4*>(x + base);
  const float4* r4 = reinterpret_cast<const float4*>(r + base);
  float4* p4 = reinterpret_cast<float4*>(p + base);
  const uint2* m4 = reinterpret_cast<const uint2*>(m + base);
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride) {
    const float4 rv = ld_nt(r4 + i);
    const float4 mv = ld_bf4(m4 + i);
    // lattice coordinates of the four elements
    const unsigned j = 4u * (unsigned)i;
    const unsigned t = j / (unsigned)f.PX;
    int xp = (int)(j - t * (unsigned)f.PX);
    int zp = (int)(t / (unsigned)f.PY);
    int yp = (int)t - zp * f.PY;
    float cz[4];
    for (int e = 0; e < 4; ++e) {
      const int xx = xp - 1, yy = yp - 1, zz = zp - 1;
      cz[e] = (xx >= 0 && xx < fx && yy >= 0 && yy < fy && zz >= 0 && zz < fz)
                  ? zs[((long long)(zz >> 1) * ey1 + (yy >> 1)) * ex1 + (xx >> 1)]
                  : 0.f;
      if (++xp == f.PX) { xp = 0; if (++yp == f.PY) { yp = 0; ++zp; } }
    }
    float4 z;
    z.x = __fmaf_rn(omega_f * mv.x, rv.x, cz[0]);
    z.y = __fmaf_rn(omega_f * mv.y, rv.y, cz[1]);
    z.z = __fmaf_rn(omega_f * mv.z, rv.z, cz[2]);
    z.w = __fmaf_rn(omega_f * mv.w, rv.w, cz[3]);
    if constexpr (OP == 2) {
      float4 pv = ld_nt(p4 + i), xv = ld_nt(x4 + i);
      xv.x = __fmaf_rn(al, pv.x, xv.x); xv.y = __fmaf_rn(al, pv.y, xv.y);
      xv.z = __fmaf_rn(al, pv.z, xv.z); xv.w = __fmaf_rn(al, pv.w, xv.w);
      pv.x = __fmaf_rn(be, pv.x, z.x); pv.y = __fmaf_rn(be, pv.y, z.y);
      pv.z = __fmaf_rn(be, pv.z, z.z); pv.w = __fmaf_rn(be, pv.w, z.w);
      st_nt(x4 + i, xv);
      st_nt(p4 + i, pv);
    } else {
      st_nt(p4 + i, z);
    }
  }
}

}  // namespace pn
