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

// The block of a 3D grid in the order x, y, z, from a linear order that gives
// each XCD a contiguous range (neighbouring z planes of a slot then share an
// L2: their halo planes are read once per XCD).
__device__ __forceinline__ int3 mg_block() {
  const int nx = gridDim.x, ny = gridDim.y;
  const int q = xcd_remap(blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z), nx * ny * gridDim.z);
  return make_int3(q % nx, (q / nx) % ny, q / (nx * ny));
}

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
// level-1 V-cycle, from zero).  A thread sums kMgRestrictPer aggregates
// kBlock apart, all 8 kMgRestrictPer loads issued before the first sum; a wave
// reads 128 consecutive fine x of each of its four (y, z) rows.  Grid:
// (blocks, slots).
constexpr int kMgRestrictPer = 2;

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
  for (int i0 = blockIdx.x * (kBlock * kMgRestrictPer) + threadIdx.x; i0 < n;
       i0 += gridDim.x * (kBlock * kMgRestrictPer)) {
    float v[kMgRestrictPer][8];
#pragma unroll
    for (int u = 0; u < kMgRestrictPer; ++u) {
      const int i = i0 + u * kBlock;
      int X = 0, Y = 0, Z = 0;
      if (i < n) mg_xyz(g1, s, i, X, Y, Z);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int x = 2 * X + (c & 1), y = 2 * Y + ((c >> 1) & 1), z = 2 * Z + (c >> 2);
        v[u][c] = (i < n && x < fe[0] && y < fe[1] && z < fe[2]) ? rs[((z + 1) * PY + (y + 1)) * PX + (x + 1)] : 0.f;
      }
    }
#pragma unroll
    for (int u = 0; u < kMgRestrictPer; ++u) {
      const int i = i0 + u * kBlock;
      if (i >= n) continue;
      int X, Y, Z;
      mg_xyz(g1, s, i, X, Y, Z);
      float acc = 0.f;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int x = 2 * X + (c & 1), y = 2 * Y + ((c >> 1) & 1), z = 2 * Z + (c >> 2);
        if (x < fe[0] && y < fe[1] && z < fe[2]) acc += v[u][c];
      }
      const long long j = g1.off[s] + i;
      r1[j] = acc;
      z1[j] = omega * acc * idg1[j];
    }
  }
}

// The aggregating down pass maps the lanes of a wave onto 16 aggregates of a
// coarse (X, Y) row-major plane, four lanes each (lane = 4 a + child, child =
// (y & 1) * 2 + (x & 1)); a lane marches its fine column through `zchunk`
// coarse planes (2 zchunk fine planes), keeping z and the -z face weight of
// the plane below in registers, and each coarse plane's 2 x 2 x 2 sum closes
// with the shuffles ^1 (x partner) and ^2 (y partner), for any extents.
// Grid: (blocks of 64 aggregates of the largest coarse plane, chunks of
// coarse z planes of the deepest slot, slots), taken XCD-contiguous.
constexpr int kMgAggLanes = 4;

__device__ __forceinline__ float mg_quad_sum(float v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  return v;
}

// Down the V-cycle at level L (z_L = omega r_L / diag already formed):
// r_{L+1} = P^T (r_L - A_L z_L) and the first sweep of level L + 1, z_{L+1} =
// omega r_{L+1} / diag.
static __global__ void __launch_bounds__(kBlock) k_mg_down(const MgGeom gf, const MgGeom gc,
                                                           const float4* __restrict__ op, const float* __restrict__ r,
                                                           const float* __restrict__ zl,
                                                           const float* __restrict__ idgc, float* __restrict__ rc,
                                                           float* __restrict__ zc, float omega, int zchunk,
                                                           const DevState* __restrict__ st) {
  if (st->stop) return;
  const int3 bk = mg_block();
  const int s = bk.z, Z0 = bk.y * zchunk;
  const int fx = gf.ext[s][0], fy = gf.ext[s][1], fz = gf.ext[s][2];
  const int cx = gc.ext[s][0], na = cx * gc.ext[s][1], cz = gc.ext[s][2];
  const int t = bk.x * kBlock + threadIdx.x;
  const int a = t / kMgAggLanes, ch = t % kMgAggLanes;
  const int Y = a / cx, X = a - Y * cx;
  const int x = 2 * X + (ch & 1), y = 2 * Y + (ch >> 1);
  const bool in = a < na && x < fx && y < fy;
  const int plane = fx * fy;
  float zm = 0.f, wm = 0.f, zp = 0.f;  // z of the planes z - 1 and z, the +z weight of plane z - 1
  if (in && 2 * Z0 < fz) {
    const long long j0 = mg_at(gf, s, x, y, 2 * Z0);
    if (Z0 >= 1) {
      zm = zl[j0 - plane];
      wm = op[j0 - plane].w;
    }
    zp = zl[j0];
  }
  for (int Z = Z0; Z < Z0 + zchunk; ++Z) {  // uniform over the wave (the shuffles)
    float acc = 0.f;
    if (in) {
      for (int z = 2 * Z; z < 2 * Z + 2 && z < fz; ++z) {
        const long long j = mg_at(gf, s, x, y, z);
        const float4 o = op[j];
        const float zn = z + 1 < fz ? zl[j + plane] : 0.f;
        float od = 0.f;
        if (x + 1 < fx) od -= o.y * zl[j + 1];
        if (y + 1 < fy) od -= o.z * zl[j + fx];
        if (z + 1 < fz) od -= o.w * zn;
        if (x >= 1) od -= op[j - 1].y * zl[j - 1];
        if (y >= 1) od -= op[j - fx].z * zl[j - fx];
        if (z >= 1) od -= wm * zm;
        acc += r[j] - (o.x * zp + od);
        zm = zp;
        zp = zn;
        wm = o.w;
      }
    }
    acc = mg_quad_sum(acc);
    if (ch == 0 && a < na && Z < cz) {
      const long long jc = mg_at(gc, s, X, Y, Z);
      rc[jc] = acc;
      zc[jc] = omega * acc * idgc[jc];
    }
  }
}

// Up the V-cycle at level L: z' = z_L + P z_{L+1}, then one damped Jacobi
// sweep z'' = z' + omega (r_L - A_L z') / diag into zo.  A thread marches one
// (x, y) column through `zchunk` z planes, keeping z' and the -z face weight
// of the plane below in registers.  With `partials`, also the block sums of
// <r_L, z''> (level 1: the coarse part of <r, B r>).  Grid: (blocks of the
// largest (x, y) plane, z chunks of the deepest slot, slots), taken
// XCD-contiguous.

static __global__ void __launch_bounds__(kBlock) k_mg_up(const MgGeom gf, const MgGeom gc,
                                                         const float4* __restrict__ op, const float* __restrict__ r,
                                                         const float* __restrict__ zl, const float* __restrict__ zc,
                                                         float* __restrict__ zo, float omega, int zchunk,
                                                         double* __restrict__ partials,
                                                         const DevState* __restrict__ st) {
  if (st->stop) return;
  const int3 bk = mg_block();
  const int s = bk.z;
  const int ex = gf.ext[s][0], ey = gf.ext[s][1], ez = gf.ext[s][2];
  const int col = bk.x * kBlock + threadIdx.x;
  const int y = col / ex, x = col - y * ex;
  const int z0 = bk.y * zchunk;
  auto zf = [&](int xx, int yy, int zz) {
    return zl[mg_at(gf, s, xx, yy, zz)] + zc[mg_at(gc, s, xx >> 1, yy >> 1, zz >> 1)];
  };
  double s0 = 0.0;
  if (y < ey && z0 < ez) {
    const int z1 = min(z0 + zchunk, ez);
    float zm = 0.f, wm = 0.f;  // z' and the +z weight of plane z - 1
    if (z0 >= 1) {
      zm = zf(x, y, z0 - 1);
      wm = op[mg_at(gf, s, x, y, z0 - 1)].w;
    }
    float zp = zf(x, y, z0);
    for (int z = z0; z < z1; ++z) {
      const long long j = mg_at(gf, s, x, y, z);
      const float4 o = op[j];
      const float zn = z + 1 < ez ? zf(x, y, z + 1) : 0.f;
      float acc = 0.f;
      if (x + 1 < ex) acc -= o.y * zf(x + 1, y, z);
      if (y + 1 < ey) acc -= o.z * zf(x, y + 1, z);
      if (z + 1 < ez) acc -= o.w * zn;
      if (x >= 1) acc -= op[j - 1].y * zf(x - 1, y, z);
      if (y >= 1) acc -= op[j - ex].z * zf(x, y - 1, z);
      if (z >= 1) acc -= wm * zm;
      const float rv = r[j];
      const float out = zp + omega * (rv - (o.x * zp + acc)) * mg_rcp(o.x);
      zo[j] = out;
      s0 += (double)(rv * out);
      zm = zp;
      zp = zn;
      wm = o.w;
    }
  }
  if (partials) {
    double unused = 0.0;
    block_sum2(s0, unused);
    if (threadIdx.x == 0) {
      const int b = (bk.z * gridDim.y + bk.y) * gridDim.x + bk.x;
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

// The small levels L0..Lc of the V-cycle in one launch: block s holds slot s
// of every level from L0 in LDS (r_L and z_L of each level, then a scratch
// array of the size of level L0 + 1), takes r_L0 and z_L0 = omega r_L0 / diag
// from the kernels before, and runs the same steps as k_mg_down,
// k_mg_coarsest and k_mg_up in the same arithmetic order (a thread issues the
// operator loads of a group of its points before using any, the level data
// being in LDS, so a pass waits on global memory about once): the down passes to
// Lc, `sweeps` - 1 further sweeps there, the up passes back to L0, whose
// result goes to zout.  With `partials` (L0 = 1), partials[2 s] = <r_1, z''>
// over the slot.  Grid: (slots); kMgTailLds bounds what one slot may need.
constexpr int kMgTailLds = 15360;
constexpr int kMgTailPer = 4;  // points per thread whose operator loads are issued together

__device__ __forceinline__ int mg_tail_points(const MgTail* t, int L, int s) {
  return t->g[L].ext[s][0] * t->g[L].ext[s][1] * t->g[L].ext[s][2];
}

static __global__ void __launch_bounds__(kFinBlock) k_mg_tail(const MgTail* __restrict__ t,
                                                              const float* __restrict__ r0,
                                                              const float* __restrict__ z0,
                                                              float* __restrict__ zout, int sweeps, float omega,
                                                              double* __restrict__ partials,
                                                              const DevState* __restrict__ st) {
  __shared__ float lds[kMgTailLds];
  __shared__ double red[kFinBlock / 64];
  if (st->stop) return;
  const int s = blockIdx.x, tid = threadIdx.x, nth = blockDim.x;
  const int L0 = t->L0, Lc = t->Lc;
  auto base = [&](int L) {  // r_L at base(L), z_L after it; the scratch at base(Lc + 1)
    int o = 0;
    for (int l = L0; l < L; ++l) o += 2 * mg_tail_points(t, l, s);
    return o;
  };
  {
    const int n = mg_tail_points(t, L0, s);
    const long long off = t->g[L0].off[s];
    float* rl = lds + base(L0);
    for (int i0 = tid; i0 < n; i0 += kMgTailPer * nth) {
      float rv[kMgTailPer], zv[kMgTailPer];
#pragma unroll
      for (int u = 0; u < kMgTailPer; ++u) {
        const int i = i0 + u * nth;
        rv[u] = i < n ? r0[off + i] : 0.f;
        zv[u] = i < n ? z0[off + i] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < kMgTailPer; ++u) {
        const int i = i0 + u * nth;
        if (i < n) { rl[i] = rv[u]; rl[n + i] = zv[u]; }
      }
    }
  }
  __syncthreads();
  // down: r_{L+1} = P^T (r_L - A_L z_L), z_{L+1} = omega r_{L+1} / diag
  for (int L = L0; L < Lc; ++L) {
    const MgGeom& gf = t->g[L];
    const MgGeom& gc = t->g[L + 1];
    const int fx = gf.ext[s][0], fy = gf.ext[s][1], fz = gf.ext[s][2];
    const int cx = gc.ext[s][0], cy = gc.ext[s][1];
    const int nf = fx * fy * fz, nc = cx * cy * gc.ext[s][2];
    const float* rl = lds + base(L);
    const float* zl = rl + nf;
    float* rc = lds + base(L + 1);
    float* zc = rc + nc;
    const float4* op = t->op[L] + gf.off[s];
    const float* idgc = t->idg[L + 1] + gc.off[s];
    for (int I = tid; I < nc; I += nth) {
      const int X = I % cx, Y = (I / cx) % cy, Z = I / (cx * cy);
      // the operator entries of the 8 children (own and the -x, -y, -z face
      // weights), all loads in flight before the first use
      float4 o[8];
      float wm[8][3];
#pragma unroll
      for (int c8 = 0; c8 < 8; ++c8) {
        const int x = 2 * X + (c8 & 1), y = 2 * Y + ((c8 >> 1) & 1), z = 2 * Z + (c8 >> 2);
        const bool in = x < fx && y < fy && z < fz;
        const int j = (z * fy + y) * fx + x;
        o[c8] = in ? op[j] : make_float4(1.f, 0.f, 0.f, 0.f);
        wm[c8][0] = in && x >= 1 ? op[j - 1].y : 0.f;
        wm[c8][1] = in && y >= 1 ? op[j - fx].z : 0.f;
        wm[c8][2] = in && z >= 1 ? op[j - fx * fy].w : 0.f;
      }
      float a[4];
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) {
        const int x = 2 * X + (ch & 1), y = 2 * Y + (ch >> 1);
        float acc = 0.f;
        if (x < fx && y < fy) {
#pragma unroll
          for (int dz = 0; dz < 2; ++dz) {
            const int z = 2 * Z + dz;
            if (z < fz) {
              const int c8 = ch + 4 * dz;
              const int j = (z * fy + y) * fx + x;
              const float4 oo = o[c8];
              float od = 0.f;
              if (x + 1 < fx) od -= oo.y * zl[j + 1];
              if (y + 1 < fy) od -= oo.z * zl[j + fx];
              if (z + 1 < fz) od -= oo.w * zl[j + fx * fy];
              if (x >= 1) od -= wm[c8][0] * zl[j - 1];
              if (y >= 1) od -= wm[c8][1] * zl[j - fx];
              if (z >= 1) od -= wm[c8][2] * zl[j - fx * fy];
              acc += rl[j] - (oo.x * zl[j] + od);
            }
          }
        }
        a[ch] = acc;
      }
      const float v = (a[0] + a[1]) + (a[2] + a[3]);
      rc[I] = v;
      zc[I] = omega * v * idgc[I];
    }
    __syncthreads();
  }
  // coarsest: sweeps 2..`sweeps` of damped Jacobi, ping-pong with the scratch
  float* zfin;
  {
    const MgGeom& g = t->g[Lc];
    const int ex = g.ext[s][0], ey = g.ext[s][1], ez = g.ext[s][2];
    const int n = ex * ey * ez;
    const float* rl = lds + base(Lc);
    float* cur = lds + base(Lc) + n;
    float* nxt = lds + base(Lc + 1);
    const float4* op = t->op[Lc] + g.off[s];
    int nb[kMgCoarsePer][6];
    float w[kMgCoarsePer][6], dg[kMgCoarsePer], idg[kMgCoarsePer], rv[kMgCoarsePer];
    for (int u = 0; u < kMgCoarsePer; ++u) {
      const int i = tid + u * nth;
      dg[u] = 1.f; idg[u] = 0.f; rv[u] = 0.f;
      for (int e = 0; e < 6; ++e) { nb[u][e] = 0; w[u][e] = 0.f; }
      if (i >= n) continue;
      const int c3[3] = {i % ex, (i / ex) % ey, i / (ex * ey)};
      const int e3[3] = {ex, ey, ez};
      const float4 o = op[i];
      const float wp[3] = {o.y, o.z, o.w};
      dg[u] = o.x;
      idg[u] = mg_rcp(o.x);
      rv[u] = rl[i];
      for (int d = 0; d < 3; ++d) {
        const int stride = d == 0 ? 1 : (d == 1 ? ex : ex * ey);
        nb[u][2 * d] = i; nb[u][2 * d + 1] = i;
        if (c3[d] + 1 < e3[d]) { nb[u][2 * d] = i + stride; w[u][2 * d] = wp[d]; }
        if (c3[d] >= 1) {
          const float4 om = op[i - stride];
          nb[u][2 * d + 1] = i - stride;
          w[u][2 * d + 1] = d == 0 ? om.y : (d == 1 ? om.z : om.w);
        }
      }
    }
    for (int sw = 1; sw < sweeps; ++sw) {
      for (int u = 0; u < kMgCoarsePer; ++u) {
        const int i = tid + u * nth;
        if (i >= n) continue;
        float az = dg[u] * cur[i];
        for (int e = 0; e < 6; ++e) az -= w[u][e] * cur[nb[u][e]];
        nxt[i] = cur[i] + omega * (rv[u] - az) * idg[u];
      }
      __syncthreads();
      float* tmp = cur;
      cur = nxt;
      nxt = tmp;
    }
    zfin = cur;
  }
  // up: z' = z_L + P z_{L+1} in place, then z'' = z' + omega (r_L - A_L z') / diag
  double s0 = 0.0;
  for (int L = Lc - 1; L >= L0; --L) {
    const MgGeom& gf = t->g[L];
    const int ex = gf.ext[s][0], ey = gf.ext[s][1], ez = gf.ext[s][2];
    const int cx = t->g[L + 1].ext[s][0], cy = t->g[L + 1].ext[s][1];
    const int n = ex * ey * ez;
    const float* rl = lds + base(L);
    float* zl = lds + base(L) + n;
    for (int i = tid; i < n; i += nth) {
      const int x = i % ex, y = (i / ex) % ey, z = i / (ex * ey);
      zl[i] = zl[i] + zfin[((z >> 1) * cy + (y >> 1)) * cx + (x >> 1)];
    }
    __syncthreads();
    float* out = lds + base(Lc + 1);
    const float4* op = t->op[L] + gf.off[s];
    for (int i0 = tid; i0 < n; i0 += kMgTailPer * nth) {
      float4 o[kMgTailPer];
      float wm[kMgTailPer][3];
#pragma unroll
      for (int u = 0; u < kMgTailPer; ++u) {
        const int i = i0 + u * nth;
        const int x = i % ex, y = (i / ex) % ey, z = i / (ex * ey);
        const bool in = i < n;
        o[u] = in ? op[i] : make_float4(1.f, 0.f, 0.f, 0.f);
        wm[u][0] = in && x >= 1 ? op[i - 1].y : 0.f;
        wm[u][1] = in && y >= 1 ? op[i - ex].z : 0.f;
        wm[u][2] = in && z >= 1 ? op[i - ex * ey].w : 0.f;
      }
#pragma unroll
      for (int u = 0; u < kMgTailPer; ++u) {
        const int i = i0 + u * nth;
        if (i < n) {
          const int x = i % ex, y = (i / ex) % ey, z = i / (ex * ey);
          const float4 oo = o[u];
          const float zp = zl[i];
          float od = 0.f;
          if (x + 1 < ex) od -= oo.y * zl[i + 1];
          if (y + 1 < ey) od -= oo.z * zl[i + ex];
          if (z + 1 < ez) od -= oo.w * zl[i + ex * ey];
          if (x >= 1) od -= wm[u][0] * zl[i - 1];
          if (y >= 1) od -= wm[u][1] * zl[i - ex];
          if (z >= 1) od -= wm[u][2] * zl[i - ex * ey];
          const float rvi = rl[i];
          const float v = zp + omega * (rvi - (oo.x * zp + od)) * mg_rcp(oo.x);
          if (L > L0) {
            out[i] = v;
          } else {
            zout[gf.off[s] + i] = v;
            s0 += (double)(rvi * v);
          }
        }
      }
    }
    __syncthreads();
    zfin = out;
  }
  if (partials) {
    s0 = wave_sum(s0);
    if ((tid & 63) == 0) red[tid >> 6] = s0;
    __syncthreads();
    if (tid == 0) {
      double a = 0.0;
      for (int wv = 0; wv < (nth >> 6); ++wv) a += red[wv];
      partials[2 * s] = a;
      partials[2 * s + 1] = 0.0;
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
