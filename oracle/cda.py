"""Classical diffusion approximation (CDA), FP64.  ORACLE: test
infrastructure only.

Section "Results": the diffusion solver the paper compares against is the
P_1 equations collapsed onto the fluence coefficient phi = L^{0,0}:

    sigma_a phi - div( 1 / (3 sigma_t') grad phi ) = Q^{0,0},

sigma_a = (1 - albedo) sigma_t and sigma_t' = sigma_t - g sigma_s (the
collision coefficient of the l = 1 equations), with the thresholded
extinction.  Reading: the printed equation has neither the absorption term
nor the reduced extinction; the collapse of the P_1 equations keeps both
(they matter for an albedo below 1 and g != 0), and only with them does the
P_1 solution equal the CDA one, which the paper states.

Discretisation (finite volumes on the voxel grid, phi at the cell centres):
the flux through the face between neighbouring cells i and j is
D_f (phi_i - phi_j) / h, D_f = 1 / (3 sigma'_f), sigma'_f the mean of
sigma_t' over the two cells.  Boundary faces: vacuum -- the cell beyond the
face holds phi = 0 and, for sigma'_f, the values of the cell inside; Neumann
-- no flux; periodic -- the neighbour wraps.  This is the operator the
staggered P_1 system leaves on the cell centres once its face unknowns are
eliminated, which ``tests/`` checks against the assembled P_1 matrix.

Cells are numbered (z n_y + y) n_x + x, fields indexed [z, y, x].
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import cell_size
from .medium import threshold
from .stagger import BC_NEUMANN, BC_PERIODIC, bc_axes


def cda_matrix(dims, sigma_t, albedo, g, sigma_t_min, bc=0, h=None):
    """Sparse (n_cells x n_cells) CDA operator."""
    nx, ny, nz = dims
    hh = cell_size(dims, h)
    bcs = bc_axes(bc)
    st = threshold(sigma_t, sigma_t_min)
    ss = np.asarray(albedo, dtype=np.float64) * st
    sa = st - ss
    spr = st - float(np.float32(g)) * ss
    ncell = nx * ny * nz
    idx = np.arange(ncell).reshape(nz, ny, nx)
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [sa.ravel()]
    for d, ax in ((0, 2), (1, 1), (2, 0)):
        n = dims[d]
        for side in (-1, 1):
            nb = np.arange(n) + side
            inside = (nb >= 0) & (nb < n)
            if bcs[d] == BC_PERIODIC:
                nbi = np.mod(nb, n)
            else:
                nbi = np.clip(nb, 0, n - 1)
            s_nb = np.take(spr, nbi, axis=ax)
            coef = 1.0 / (3.0 * 0.5 * (spr + s_nb) * hh * hh)
            keep = np.broadcast_to(np.expand_dims(inside, tuple(a for a in range(3) if a != ax)), spr.shape)
            if bcs[d] == BC_PERIODIC:
                keep = np.ones(spr.shape, dtype=bool)
            j = np.take(idx, nbi, axis=ax)
            # diagonal: every face with a flux (inside, periodic, or vacuum boundary)
            flux = keep if bcs[d] == BC_NEUMANN else np.ones(spr.shape, dtype=bool)
            rows.append(idx[flux])
            cols.append(idx[flux])
            vals.append(coef[flux])
            rows.append(idx[keep])
            cols.append(j[keep])
            vals.append(-coef[keep])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(ncell, ncell))
    A.sum_duplicates()
    return A


def cda_solve(dims, sigma_t, albedo, g, sigma_t_min, q00, bc=0, h=None, tol=1e-13, direct_max=200000):
    """phi [z, y, x] of the CDA operator for the emission q00 [z, y, x]: SuperLU
    up to ``direct_max`` cells, above that conjugate gradients (the operator
    is symmetric positive definite) to the relative residual ``tol``."""
    A = cda_matrix(dims, sigma_t, albedo, g, sigma_t_min, bc, h)
    b = np.asarray(q00, dtype=np.float64).ravel()
    if A.shape[0] <= direct_max:
        phi = spla.splu(A.tocsc()).solve(b)
    else:
        phi, info = spla.cg(A, b, rtol=tol, atol=0.0, maxiter=100000)
        if info != 0:
            raise RuntimeError("CDA conjugate gradients did not converge")
    nx, ny, nz = dims
    return phi.reshape(nz, ny, nx)
