"""Staggered placement of the SH coefficients and the flat vector layout
(oracle; test infrastructure only).

The paper distributes the coefficients over disjoint staggered grids (section
"P_N-Solver", staggering figure) following StaRMAP and defers the placement
rule to that work.  The reading used here: a coefficient sits at the offset
(p_x, p_y, p_z) in {0,1}^3 given by the parity of Y_R^{l,m} under reflection
of each axis (1 = odd):

    p_x = m mod 2 (m >= 0),  (|m|+1) mod 2 (m < 0)
    p_y = 1 if m < 0 else 0
    p_z = (l + |m|) mod 2

A coupling int omega_d Y^k Y^k' is non-zero only if the classes of k and k'
differ in axis d and agree in the other two, so every spatial derivative in
the transport term is a two-point central difference over one cell width and
no unknown ever has to be interpolated.  ``tests/`` checks this against the
quadrature couplings rather than assuming it.

Grid: n_x * n_y * n_z cells of size h (unit cube: h = 1/n).  Along axis d a
coefficient of class p sits at (i + 1/2 - p_d/2) h:
  * vacuum (homogeneous Dirichlet) or Neumann boundary: i = 0 .. n_d - 1 + p_d,
    i.e. the face-centred classes include both boundary faces (the "additional
    coefficients at boundary voxels" of the paper's un-staggering step);
  * periodic boundary: i = 0 .. n_d - 1, indices wrap.
The boundary type may differ per axis (a 2D problem is a z-periodic grid of
one cell in z).

Boundary handling of a difference that references an index outside the
class extent (section "Runtime", last paragraph): the Dirichlet boundary
drops the entry (the value outside is 0); the Neumann boundary moves the
entry to the column of the coefficient in the closest location inside the
domain (the index is clamped into the extent); the periodic grid wraps.

Flat vector layout: coefficients in k order; the array of each coefficient is
contiguous, z-major / x-fastest over that class's extent.
"""
import numpy as np

from .sh import coeff_lm, num_coeffs

BC_VACUUM = 0
BC_PERIODIC = 1
BC_NEUMANN = 2


def bc_axes(bc):
    """Boundary types (x, y, z) from one type for every axis or a 3-sequence."""
    if isinstance(bc, (int, np.integer)):
        return (int(bc),) * 3
    t = tuple(int(b) for b in bc)
    if len(t) != 3:
        raise ValueError("bc must be one type or three")
    return t


def resolve_index(idx, ext_d, bc_d):
    """Index along one axis of an unknown that a difference references: kept
    when inside [0, ext_d); outside it is dropped (None) under the Dirichlet
    boundary, wrapped under the periodic one and moved to the closest index
    inside under the Neumann one."""
    if 0 <= idx < ext_d:
        return idx
    if bc_d == BC_PERIODIC:
        return idx % ext_d
    if bc_d == BC_NEUMANN:
        return min(max(idx, 0), ext_d - 1)
    return None


def coeff_class(l, m):
    """(p_x, p_y, p_z) of coefficient (l, m): axis parities of Y_R^{l,m}."""
    am = abs(m)
    px = (m % 2) if m >= 0 else ((am + 1) % 2)
    py = 1 if m < 0 else 0
    pz = (l + am) % 2
    return (px, py, pz)


def class_of_k(k):
    l, m = coeff_lm(k)
    return coeff_class(l, m)


def class_extent(p, dims, bc):
    """(e_x, e_y, e_z) lattice extent of class p on a grid of dims=(nx,ny,nz)."""
    b = bc_axes(bc)
    return tuple(int(dims[d]) + (0 if b[d] == BC_PERIODIC else int(p[d])) for d in range(3))


class Layout:
    """Offsets and extents of every coefficient array in the flat vector."""

    def __init__(self, order, dims, bc=BC_VACUUM):
        self.order = int(order)
        self.dims = tuple(int(v) for v in dims)
        self.bcs = bc_axes(bc)
        self.bc = self.bcs[0] if len(set(self.bcs)) == 1 else self.bcs
        self.ncoeff = num_coeffs(order)
        self.cls = [class_of_k(k) for k in range(self.ncoeff)]
        self.ext = [class_extent(self.cls[k], self.dims, self.bc) for k in range(self.ncoeff)]
        self.size = [e[0] * e[1] * e[2] for e in self.ext]
        self.offset = np.concatenate([[0], np.cumsum(self.size)]).astype(np.int64)
        self.n = int(self.offset[-1])

    def view(self, vec, k):
        """Array of coefficient k as shape (e_z, e_y, e_x) (a view into vec)."""
        ex, ey, ez = self.ext[k]
        return vec[self.offset[k]:self.offset[k + 1]].reshape(ez, ey, ex)

    def positions(self, k):
        """Physical positions (in units of h) of coefficient k's lattice points,
        as three arrays of shape (e_z, e_y, e_x)."""
        ex, ey, ez = self.ext[k]
        p = self.cls[k]
        z, y, x = np.meshgrid(np.arange(ez), np.arange(ey), np.arange(ex), indexing="ij")
        return (x + 0.5 - 0.5 * p[0], y + 0.5 - 0.5 * p[1], z + 0.5 - 0.5 * p[2])

    def flat_index(self, k, i, j, l):
        """Flat vector index of coefficient k at lattice point (i, j, l) = (x, y, z)."""
        ex, ey, _ = self.ext[k]
        return int(self.offset[k]) + (l * ey + j) * ex + i


def num_unknowns(order, dims, bc=BC_VACUUM):
    return Layout(order, dims, bc).n
