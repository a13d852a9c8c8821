"""Rendering-side operations of the P_N method (section "Rendering"), FP64.
ORACLE: test infrastructure only.

* ``unstagger``: the solution's coefficients interpolated to the voxel
  centres.  A coefficient of class p sits, along axis d, at the cell centres
  (p_d = 0: the value of the cell's own lattice point) or on the cell faces
  (p_d = 1: the mean of the two faces of the cell, i and i + 1; on a periodic
  axis face n is face 0).  The boundary coefficients beyond the cells are not
  used.  Result: [(N+1)^2, nz, ny, nx].

* ``single_scatter_source``: the single-scattered light folded into the
  emission term, Q = L_ss(x, w) = sigma_s(x) int p(w' -> w) L_u(x, w') dw',
  with L_u the uncollided light of a point light of power Phi at x_L:
  L_u(x, w') = Phi exp(-tau(x_L, x)) / (4 pi r^2) delta(w' - w_L), r = |x -
  x_L|, w_L = (x - x_L) / r the direction the light travels, tau the optical
  depth of the segment.  For the Henyey-Greenstein phase function the
  projection onto Y_R^{l,m} is int p(w_L . w) Y_R^{l,m}(w) dw = g^l Y_R^{l,m}(w_L)
  (pinned by quadrature in tests/), so
      Q^{l,m}(x) = sigma_s(x) Phi exp(-tau) / (4 pi r^2) g^l Y_R^{l,m}(w_L),
  evaluated at the location of each unknown (its staggered position), with
  sigma_s interpolated there as in ``medium`` (mean of the adjacent cells) and
  tau through the thresholded extinction of the cells, constant per cell,
  outside the domain zero (vacuum).  Readings: the paper computes L_u "using
  a few light samples per voxel"; for a point light one exact sample per
  location is used.  The distance is clamped to at least h / 2 (a location on
  the light itself).  Periodic axes are not supported (the light would have
  infinitely many images).
"""
import numpy as np

from .assemble import cell_size
from .medium import interpolate_to_class, threshold
from .sh import coeff_lm, real_sh
from .stagger import BC_PERIODIC, Layout


def unstagger(layout, u):
    """[(N+1)^2, nz, ny, nx] values at the voxel centres."""
    nx, ny, nz = layout.dims
    out = np.empty((layout.ncoeff, nz, ny, nx))
    for k in range(layout.ncoeff):
        a = layout.view(np.asarray(u, dtype=np.float64), k)  # (ez, ey, ex)
        p = layout.cls[k]
        for d, ax in ((0, 2), (1, 1), (2, 0)):
            n = layout.dims[d]
            if p[d] == 1:
                lo = np.take(a, np.arange(n), axis=ax)
                hi_idx = np.arange(1, n + 1)
                if layout.bcs[d] == BC_PERIODIC:
                    hi_idx = np.mod(hi_idx, n)
                hi = np.take(a, hi_idx, axis=ax)
                a = 0.5 * (lo + hi)
            else:
                a = np.take(a, np.arange(n), axis=ax)
        out[k] = a
    return out


def segment_optical_depth(sigma, h, p0, p1):
    """Exact optical depth of the segment p0 -> p1 through cells of size h
    with constant extinction sigma[z, y, x] each (zero outside the grid): the
    length of the segment inside every cell box, times its extinction.  Cells
    are half-open boxes [i h, (i+1) h): a segment lying in a face plane
    belongs to the cell above that face (or to none on the upper boundary)."""
    p0 = np.asarray(p0, dtype=np.float64)
    p1 = np.asarray(p1, dtype=np.float64)
    nz, ny, nx = sigma.shape
    dvec = p1 - p0
    length = float(np.linalg.norm(dvec))
    if length == 0.0:
        return 0.0
    lo = np.floor(np.minimum(p0, p1) / h).astype(int)
    hi = np.floor(np.maximum(p0, p1) / h).astype(int)
    lo = np.maximum(lo, 0)
    hi = np.minimum(hi, np.array([nx - 1, ny - 1, nz - 1]))
    tau = 0.0
    for iz in range(lo[2], hi[2] + 1):
        for iy in range(lo[1], hi[1] + 1):
            for ix in range(lo[0], hi[0] + 1):
                bmin = np.array([ix, iy, iz], dtype=np.float64) * h
                bmax = bmin + h
                t0, t1 = 0.0, 1.0
                for d in range(3):
                    if dvec[d] == 0.0:  # cells are half-open boxes [bmin, bmax)
                        if not (bmin[d] <= p0[d] < bmax[d]):
                            t0, t1 = 1.0, 0.0
                        continue
                    ta = (bmin[d] - p0[d]) / dvec[d]
                    tb = (bmax[d] - p0[d]) / dvec[d]
                    t0 = max(t0, min(ta, tb))
                    t1 = min(t1, max(ta, tb))
                if t1 > t0:
                    tau += sigma[iz, iy, ix] * (t1 - t0) * length
    return tau


def single_scatter_source(order, dims, sigma_t, albedo, g, sigma_t_min, light, power, bc=0, h=None):
    """Packed right-hand side Q^{l,m} of the single-scattered light of a point
    light at ``light`` (physical coordinates) with power ``power``."""
    lay = Layout(order, dims, bc)
    if any(b == BC_PERIODIC for b in lay.bcs):
        raise ValueError("single scattering needs a non-periodic domain")
    hh = cell_size(dims, h)
    st = threshold(sigma_t, sigma_t_min)
    ss = np.asarray(albedo, dtype=np.float64) * st
    gg = float(np.float32(g))
    light = np.asarray(light, dtype=np.float64)
    q = np.zeros(lay.n)
    cache = {}
    for k in range(lay.ncoeff):
        l, m = coeff_lm(k)
        p = lay.cls[k]
        if p not in cache:
            ex, ey, ez = lay.ext[k]
            sigs = interpolate_to_class(ss, p, lay.ext[k], lay.bcs)
            vals = np.empty((ez, ey, ex))
            theta = np.empty((ez, ey, ex))
            phi = np.empty((ez, ey, ex))
            for iz in range(ez):
                for iy in range(ey):
                    for ix in range(ex):
                        pos = (np.array([ix, iy, iz], dtype=np.float64) + 0.5 - 0.5 * np.array(p)) * hh
                        v = pos - light
                        r = max(float(np.linalg.norm(v)), 0.5 * hh)
                        tau = segment_optical_depth(st, hh, light, pos)
                        vals[iz, iy, ix] = sigs[iz, iy, ix] * power * np.exp(-tau) / (4.0 * np.pi * r * r)
                        nv = float(np.linalg.norm(v))
                        w = v / nv if nv > 0.0 else np.array([0.0, 0.0, 1.0])
                        theta[iz, iy, ix] = np.arccos(np.clip(w[2], -1.0, 1.0))
                        phi[iz, iy, ix] = np.arctan2(w[1], w[0])
            cache[p] = (vals, theta, phi)
        vals, theta, phi = cache[p]
        lay.view(q, k)[...] = vals * (gg ** l) * real_sh(l, m, theta, phi)
    return q, lay
