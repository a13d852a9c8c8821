"""Sparse FP64 assembly of the staggered real P_N system A u = Q
(oracle; test infrastructure only).

Paper, "Discretized Radiative Transfer Equation": after projection the P_N
equations are discretised with central finite differences on a voxel grid,
the coefficients of all voxels are flattened into u and the projected
operators collapse into one matrix A = T + C - S.  Section "Runtime": the
system is filled row by row; under the Dirichlet boundary condition a write to
a location outside the domain is dropped, under the Neumann boundary condition
it goes to the row and column of the coefficient in the closest location
inside the domain (the written index is changed).

Row of coefficient k (class p) at lattice point x (the real P_N equations of
section "Real-valued P_N-equations", with couplings by quadrature):

    sum_d sum_k'  A_d[k,k'] (u_k'(x + h/2 e_d) - u_k'(x - h/2 e_d)) / h
  + (sigma_t(x) - g^l sigma_s(x)) u_k(x)                          =  Q_k(x)

where k' has the class of k with axis d flipped (see ``stagger``).  In index
terms, with i the index of x along d:
  * k' face-centred along d (p'_d = 1):  u_k'[i+1] - u_k'[i]
  * k' cell-centred along d (p'_d = 0):  u_k'[i]   - u_k'[i-1]
Indices outside the class extent read 0 (vacuum), wrap (periodic) or are
clamped into the extent (Neumann); see ``stagger.resolve_index``.  Only the
cell-centred references of the boundary face rows ever leave the extent, so
under the Neumann boundary those rows lose that difference.

The cell size h defaults to 1/n_x (unit cube for cubic grids).

Two implementations are given: ``assemble_rows`` is a pure-Python loop over
rows for tiny grids; ``assemble`` builds the same matrix with vectorised index
arithmetic.  ``tests/`` checks one against the other.
"""
import numpy as np
import scipy.sparse as sp

from .couplings import coupling_list
from .medium import diagonal
from .stagger import Layout, BC_PERIODIC, BC_NEUMANN, resolve_index


def _neighbour_pair(i, pprime_d, ext_d, bc_d):
    """Indices (plus, minus) along the derivative axis after the boundary rule
    (None: the entry is dropped)."""
    if pprime_d == 1:
        ip, im = i + 1, i
    else:
        ip, im = i, i - 1
    return resolve_index(ip, ext_d, bc_d), resolve_index(im, ext_d, bc_d)


def cell_size(dims, h=None):
    """h, defaulting to 1/n_x."""
    return 1.0 / dims[0] if h is None or h <= 0 else float(h)


def assemble_rows(order, dims, sigma_t, albedo, g, sigma_t_min, bc=0, couplings=None, h=None):
    """Pure-Python, row-by-row assembly (tiny grids only). Returns (A_csr, layout)."""
    lay = Layout(order, dims, bc)
    cl = coupling_list(order) if couplings is None else couplings
    by_row = {}
    for (k, d, kp, c) in cl:
        by_row.setdefault(k, []).append((d, kp, c))
    diag = diagonal(lay, sigma_t, albedo, g, sigma_t_min)
    h = cell_size(dims, h)
    entries = {}
    for k in range(lay.ncoeff):
        ex, ey, ez = lay.ext[k]
        for z in range(ez):
            for y in range(ey):
                for x in range(ex):
                    row = lay.flat_index(k, x, y, z)
                    entries[(row, row)] = entries.get((row, row), 0.0) + diag[k][z, y, x]
                    for (d, kp, c) in by_row.get(k, []):
                        pt = [x, y, z]
                        ip, im = _neighbour_pair(pt[d], lay.cls[kp][d], lay.ext[kp][d], lay.bcs[d])
                        for idx, sgn in ((ip, 1.0), (im, -1.0)):
                            if idx is None:
                                continue
                            q = list(pt)
                            q[d] = idx
                            col = lay.flat_index(kp, q[0], q[1], q[2])
                            entries[(row, col)] = entries.get((row, col), 0.0) + sgn * c / h
    rows = np.array([rc[0] for rc in entries], dtype=np.int64)
    cols = np.array([rc[1] for rc in entries], dtype=np.int64)
    vals = np.array(list(entries.values()))
    return sp.csr_matrix((vals, (rows, cols)), shape=(lay.n, lay.n)), lay


def assemble(order, dims, sigma_t, albedo, g, sigma_t_min, bc=0, couplings=None, h=None):
    """Vectorised assembly of the same matrix. Returns (A_csr, layout).

    ``dims`` = (nx, ny, nz); the cell size h defaults to 1/nx (unit cube for
    cubic grids).  ``sigma_t`` and ``albedo`` are cell-centred arrays
    (nz, ny, nx).  ``bc``: one boundary type or one per axis.
    """
    lay = Layout(order, dims, bc)
    cl = coupling_list(order) if couplings is None else couplings
    diag = diagonal(lay, sigma_t, albedo, g, sigma_t_min)
    h = cell_size(dims, h)
    R, C, V = [], [], []
    for k in range(lay.ncoeff):
        rows = np.arange(lay.offset[k], lay.offset[k + 1])
        R.append(rows)
        C.append(rows)
        V.append(diag[k].ravel())
    for (k, d, kp, c) in cl:
        ex, ey, ez = lay.ext[k]
        z, y, x = np.meshgrid(np.arange(ez), np.arange(ey), np.arange(ex), indexing="ij")
        pt = [x.ravel(), y.ravel(), z.ravel()]
        rows = lay.offset[k] + (pt[2] * ey + pt[1]) * ex + pt[0]
        pe = lay.ext[kp]
        i = pt[d]
        if lay.cls[kp][d] == 1:
            ip, im = i + 1, i
        else:
            ip, im = i, i - 1
        for idx, sgn in ((ip, 1.0), (im, -1.0)):
            q = list(pt)
            if lay.bcs[d] == BC_PERIODIC:
                q[d] = np.mod(idx, pe[d])
                keep = np.ones(idx.shape, dtype=bool)
            elif lay.bcs[d] == BC_NEUMANN:
                q[d] = np.clip(idx, 0, pe[d] - 1)
                keep = np.ones(idx.shape, dtype=bool)
            else:
                keep = (idx >= 0) & (idx < pe[d])
                q[d] = idx
            cols = lay.offset[kp] + (q[2] * pe[1] + q[1]) * pe[0] + q[0]
            R.append(rows[keep])
            C.append(cols[keep])
            V.append(np.full(int(keep.sum()), sgn * c / h))
    A = sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))), shape=(lay.n, lay.n))
    A.sum_duplicates()
    return A, lay


def rhs_isotropic(layout, q00):
    """RHS vector for an isotropic emission given as Q^{0,0} per cell.

    Q^{0,0} lives at the cell centres, where coefficient k = 0 sits; every other
    Q^{l,m} of an isotropic source is zero (section "Real-valued
    P_N-equations": the emission term projects onto Q^{l,m})."""
    b = np.zeros(layout.n)
    layout.view(b, 0)[...] = np.asarray(q00, dtype=np.float64)
    return b
