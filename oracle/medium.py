"""RTE parameters at the staggered locations (oracle; test infrastructure only).

* Extinction threshold (section "Runtime" and the nebulae results): every cell
  whose sigma_t is below sigma_t_min is set to sigma_t_min, because vacuum makes
  A singular.  Scattering is sigma_s = albedo * sigma_t of the thresholded value.
* RTE parameters live at cell centres; where a row sits elsewhere the solver
  interpolates them to the row location (section "Precomputation", staggered
  interpolation).  Reading: the arithmetic mean of the 1/2/4/8 cells adjacent
  to the location, cell indices clamped into the domain (vacuum boundary) or
  wrapped (periodic); the Neumann boundary clamps like the vacuum one (the
  closest cell inside the domain).  sigma_t and sigma_s are interpolated
  separately.
* The per-band diagonal (collision minus scattering, appendix "Collision term"
  and "Scattering term"):  sigma_t - sigma_s * lambda_l p^{l,0}, and for a
  Henyey-Greenstein phase function lambda_l p^{l,0} = g^l (pinned in
  ``couplings.scattering_factors``).

All arithmetic is FP64; the inputs (fields, g, sigma_t_min) are FP32 values,
rounded once from whatever the caller passes.
"""
import numpy as np

from .sh import coeff_lm
from .stagger import BC_PERIODIC, bc_axes


def threshold(sigma_t, sigma_t_min):
    """max(sigma_t, sigma_t_min) cell by cell, in FP64.  The threshold is an
    FP32 input like the fields, so it is rounded to FP32 first."""
    return np.maximum(np.asarray(sigma_t, dtype=np.float64), float(np.float32(sigma_t_min)))


def interpolate_to_class(field, p, ext, bc):
    """Mean of ``field`` (cell-centred, shape (nz, ny, nx)) over the cells
    adjacent to every lattice point of class p (extent ext = (ex, ey, ez)).

    Along axis d a class with p_d = 0 sits at a cell centre (one cell); with
    p_d = 1 it sits on the face between cells i-1 and i (two cells).
    """
    f = np.asarray(field, dtype=np.float64)
    nz, ny, nx = f.shape
    n = (nx, ny, nz)
    bcs = bc_axes(bc)
    idx = []
    for d in range(3):
        i = np.arange(ext[d])
        if p[d] == 0:
            cand = [i]
        else:
            cand = [i - 1, i]
        fixed = []
        for c in cand:
            if bcs[d] == BC_PERIODIC:
                fixed.append(np.mod(c, n[d]))
            else:
                fixed.append(np.clip(c, 0, n[d] - 1))
        idx.append(fixed)
    out = np.zeros((ext[2], ext[1], ext[0]))
    cnt = 0
    for iz in idx[2]:
        for iy in idx[1]:
            for ix in idx[0]:
                out += f[np.ix_(iz, iy, ix)]
                cnt += 1
    return out / cnt


def diagonal(layout, sigma_t, albedo, g, sigma_t_min):
    """Per-coefficient diagonal arrays  sigma_t(x_k) - g^l sigma_s(x_k).

    Returns a list indexed by k of arrays shaped like ``layout.view(., k)``.
    """
    st = threshold(sigma_t, sigma_t_min)
    ss = np.asarray(albedo, dtype=np.float64) * st
    g = float(np.float32(g))  # an FP32 input, like the fields
    cache = {}
    out = []
    for k in range(layout.ncoeff):
        l, _ = coeff_lm(k)
        p = layout.cls[k]
        if p not in cache:
            cache[p] = (interpolate_to_class(st, p, layout.ext[k], layout.bcs),
                        interpolate_to_class(ss, p, layout.ext[k], layout.bcs))
        t, s = cache[p]
        out.append(t - (float(g) ** l) * s)
    return out
