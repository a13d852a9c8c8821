// Rendering-side kernels of the P_N method (section "Rendering"): the
// single-scattered light of a point light folded into the emission term, and
// the un-staggering of a solution to the voxel centres.
#pragma once
#include <hip/hip_runtime.h>

#include "pn_kernels.h"

namespace pn {

// Geometry of the packed (API) layout and the padded medium.
struct RenderArgs {
  int nc, nx, ny, nz;
  int per[3];                 // periodic axes (un-staggering only)
  long long off[kMaxCoeff];   // packed offsets
  int ext[kMaxCoeff][3];      // class extents (ex, ey, ez)
  int cls[kMaxCoeff][3];      // staggering class
  double h;
  double light[3];            // physical position of the point light
  double power;
  double g;                   // Henyey-Greenstein mean cosine (as FP32 input, widened)
  const float2* med;          // padded cells (sigma_t thresholded, albedo)
};

__device__ __forceinline__ long long med_index(const RenderArgs& a, int x, int y, int z) {
  return ((long long)(z + 1) * (a.ny + 2) + (y + 1)) * (a.nx + 2) + (x + 1);
}

// Real spherical harmonic Y_R^{l,m} (the basis of section "Real-valued
// P_N-equations" / appendix): with mu = |m| and P^{l,mu} the associated
// Legendre function without the Condon-Shortley phase,
//   m < 0: sqrt 2 K P^{l,mu}(cos t) sin(mu p), m = 0: K P^{l,0}(cos t),
//   m > 0: sqrt 2 K P^{l,m}(cos t) cos(m p),
// K = sqrt((2l + 1) / (4 pi) (l - mu)! / (l + mu)!).  Direction (wx, wy, wz) of
// unit length: cos t = wz, p = atan2(wy, wx).
__device__ inline double real_sh_dir(int l, int m, double wx, double wy, double wz) {
  const int mu = m < 0 ? -m : m;
  const double ct = wz, st = sqrt(fmax(0.0, 1.0 - wz * wz));
  // P^{mu,mu} = (2 mu - 1)!! st^mu, then the three-term recurrence in l
  double pmm = 1.0;
  for (int i = 1; i <= mu; ++i) pmm *= (2.0 * i - 1.0) * st;
  double plm = pmm;
  if (l > mu) {
    double p0 = pmm, p1 = ct * (2.0 * mu + 1.0) * pmm;
    for (int ll = mu + 2; ll <= l; ++ll) {
      const double p2 = ((2.0 * ll - 1.0) * ct * p1 - (ll + mu - 1.0) * p0) / (ll - mu);
      p0 = p1;
      p1 = p2;
    }
    plm = p1;
  }
  double ratio = 1.0;  // (l - mu)! / (l + mu)!
  for (int i = l - mu + 1; i <= l + mu; ++i) ratio /= (double)i;
  const double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * ratio);
  if (m == 0) return K * plm;
  const double phi = atan2(wy, wx);
  return sqrt(2.0) * K * plm * (m > 0 ? cos(mu * phi) : sin(mu * phi));
}

// Optical depth of the segment p0 -> p1 through the cells (extinction
// constant per cell, zero outside the grid): the segment is clipped to the
// grid box and walked cell by cell (the 3D digital differential analyser of
// Amanatides & Woo), each cell contributing its extinction times the length
// of the segment inside it.  Cells are half-open boxes [i h, (i+1) h), so a
// segment lying in a face plane belongs to the cell above it.  At most
// nx + ny + nz + 3 steps.
__device__ inline double optical_depth(const RenderArgs& a, const double* p0, const double* p1) {
#pragma clang fp contract(off)
  const double d[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
  const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  if (len == 0.0) return 0.0;
  const int n[3] = {a.nx, a.ny, a.nz};
  double t0 = 0.0, t1 = 1.0;
  for (int k = 0; k < 3; ++k) {
    const double bmax = n[k] * a.h;
    if (d[k] == 0.0) {  // cells are half-open boxes [i h, (i+1) h)
      if (p0[k] < 0.0 || p0[k] >= bmax) return 0.0;
      continue;
    }
    const double ta = (0.0 - p0[k]) / d[k], tb = (bmax - p0[k]) / d[k];
    t0 = fmax(t0, fmin(ta, tb));
    t1 = fmin(t1, fmax(ta, tb));
  }
  if (!(t1 > t0)) return 0.0;
  int c[3], step[3];
  double tmax[3], tdelta[3];
  const double tm = 0.5 * (t0 + t1);  // a point inside the clipped segment picks the start cell robustly
  for (int k = 0; k < 3; ++k) {
    const double s = p0[k] + t0 * d[k];
    int ci = (int)floor(s / a.h);
    if (d[k] > 0.0 && ci >= n[k]) ci = n[k] - 1;
    if (d[k] < 0.0 && s == ci * a.h) ci -= 1;  // leaving a face backwards: the cell below it
    if (d[k] == 0.0) ci = (int)floor((p0[k] + tm * d[k]) / a.h);
    c[k] = min(max(ci, 0), n[k] - 1);
    if (d[k] > 0.0) {
      step[k] = 1;
      tmax[k] = ((c[k] + 1) * a.h - p0[k]) / d[k];
      tdelta[k] = a.h / d[k];
    } else if (d[k] < 0.0) {
      step[k] = -1;
      tmax[k] = (c[k] * a.h - p0[k]) / d[k];
      tdelta[k] = -a.h / d[k];
    } else {
      step[k] = 0;
      tmax[k] = 2.0;
      tdelta[k] = 2.0;
    }
  }
  double tau = 0.0, t = t0;
  const int maxsteps = a.nx + a.ny + a.nz + 3;
  for (int it = 0; it < maxsteps; ++it) {
    int ax = 0;
    if (tmax[1] < tmax[ax]) ax = 1;
    if (tmax[2] < tmax[ax]) ax = 2;
    const double tn = fmin(tmax[ax], t1);
    if (tn > t) tau += (double)a.med[med_index(a, c[0], c[1], c[2])].x * (tn - t) * len;
    t = tn;
    if (t >= t1) break;
    c[ax] += step[ax];
    if (c[ax] < 0 || c[ax] >= n[ax]) break;
    tmax[ax] += tdelta[ax];
  }
  return tau;
}

// Q^{l,m} at every unknown (packed FP32, one thread per unknown of
// coefficient blockIdx.y): sigma_s (mean of the adjacent cells) Phi
// exp(-tau) / (4 pi r^2) g^l Y_R^{l,m}(w_L), w_L the direction from the light
// to the unknown's location, r clamped to at least h / 2.
static __global__ void __launch_bounds__(kBlock) k_single_scatter(const RenderArgs a, float* __restrict__ q) {
  // Positions and differences are rounded separately (no fused multiply-add),
  // so a location that coincides with the light gives exactly r = 0.
#pragma clang fp contract(off)
  const int k = blockIdx.y;
  const int ex = a.ext[k][0], ey = a.ext[k][1], ez = a.ext[k][2];
  const long long sz = (long long)ex * ey * ez;
  int l = 0;
  while ((l + 1) * (l + 1) <= k) ++l;
  const int m = k - l * l - l;
  const int px = a.cls[k][0], py = a.cls[k][1], pz = a.cls[k][2];
  double gl = 1.0;
  for (int i = 0; i < l; ++i) gl *= a.g;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < sz; i += (long long)gridDim.x * kBlock) {
    const int x = (int)(i % ex);
    const int y = (int)((i / ex) % ey);
    const int z = (int)(i / ((long long)ex * ey));
    // sigma_s: mean over the cells adjacent to the location (the padded
    // halo holds clamped copies)
    double ss = 0.0;
    int cnt = 0;
    for (int dz = pz ? -1 : 0; dz <= 0; ++dz)
      for (int dy = py ? -1 : 0; dy <= 0; ++dy)
        for (int dx = px ? -1 : 0; dx <= 0; ++dx) {
          const float2 c = a.med[med_index(a, x + dx, y + dy, z + dz)];
          ss += (double)c.x * (double)c.y;
          ++cnt;
        }
    ss /= cnt;
    const double pos[3] = {(x + 0.5 - 0.5 * px) * a.h, (y + 0.5 - 0.5 * py) * a.h, (z + 0.5 - 0.5 * pz) * a.h};
    const double v[3] = {pos[0] - a.light[0], pos[1] - a.light[1], pos[2] - a.light[2]};
    const double dist = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double r = fmax(dist, 0.5 * a.h);
    const double tau = optical_depth(a, a.light, pos);
    double wx = 0.0, wy = 0.0, wz = 1.0;
    if (dist > 0.0) { wx = v[0] / dist; wy = v[1] / dist; wz = v[2] / dist; }
    const double val = ss * a.power * exp(-tau) / (4.0 * M_PI * r * r) * gl * real_sh_dir(l, m, wx, wy, wz);
    q[a.off[k] + i] = (float)val;
  }
}

// out[k][z][y][x] (FP32): coefficient k interpolated to the voxel centre --
// its own lattice point along a centred axis, the mean of the cell's two
// faces along a face axis (face n is face 0 on a periodic axis).
static __global__ void __launch_bounds__(kBlock) k_unstagger(const RenderArgs a, const double* __restrict__ u,
                                                             float* __restrict__ out) {
  const int k = blockIdx.y;
  const long long cells = (long long)a.nx * a.ny * a.nz;
  const int ex = a.ext[k][0], ey = a.ext[k][1];
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < cells; i += (long long)gridDim.x * kBlock) {
    const int x = (int)(i % a.nx);
    const int y = (int)((i / a.nx) % a.ny);
    const int z = (int)(i / ((long long)a.nx * a.ny));
    double s = 0.0;
    int cnt = 0;
    for (int dz = 0; dz <= a.cls[k][2]; ++dz)
      for (int dy = 0; dy <= a.cls[k][1]; ++dy)
        for (int dx = 0; dx <= a.cls[k][0]; ++dx) {
          int xx = x + dx, yy = y + dy, zz = z + dz;
          if (a.per[0] && xx == a.nx) xx = 0;
          if (a.per[1] && yy == a.ny) yy = 0;
          if (a.per[2] && zz == a.nz) zz = 0;
          s += u[a.off[k] + ((long long)zz * ey + yy) * ex + xx];
          ++cnt;
        }
    out[(long long)k * cells + i] = (float)(s / cnt);
  }
}

}  // namespace pn
