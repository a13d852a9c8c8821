"""Pins of the oracle's boundary handling, per-axis boundary types, cell size
and the one-row-at-a-time checker ``rows_of``.  CPU only.

Neumann boundary (section "Runtime", last paragraph): an entry that would
reference a location outside the domain is moved to the coefficient in the
closest location inside.  Pinned here by what that rule implies, not by
re-stating it:
  * a uniform medium with uniform isotropic emission has the spatially
    constant solution L00 = Q / sigma_a (no leakage through the boundary);
  * the boundary is a mirror: the solution on n cells equals the solution of
    the periodic problem on 2n cells with the medium and source reflected
    about the boundary plane (the cell-centred coefficients are even about
    the plane, the face coefficients on it vanish).
"""
from math import pi

import numpy as np
import pytest

from oracle.apply import Operator, rows_of
from oracle.assemble import assemble, assemble_rows, rhs_isotropic
from oracle.couplings import transport_couplings
from oracle import sh
from oracle.solve import direct
from oracle.stagger import BC_NEUMANN, BC_PERIODIC, BC_VACUUM, Layout
from synth import config_small

BCS = [BC_VACUUM, BC_PERIODIC, BC_NEUMANN, (BC_NEUMANN, BC_VACUUM, BC_PERIODIC), (BC_PERIODIC, BC_NEUMANN, BC_VACUUM)]


def _medium(order, dims, bc, seed=3):
    return config_small(order, dims, seed=seed, bc=bc)


# ------------------------------------------------------------- rows_of ----
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("order", [1, 3, 4])
def test_rows_of_equals_assembled_matrix_on_every_row(order, bc):
    m = _medium(order, (4, 3, 5), bc)
    A, lay = assemble(order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc)
    x = np.random.default_rng(2).normal(size=lay.n)
    rows = np.arange(lay.n)  # every row, boundary rows included
    got = rows_of(order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, x, rows, bc=bc)
    np.testing.assert_allclose(got, A @ x, rtol=1e-13, atol=1e-11)


@pytest.mark.parametrize("bc", [BC_VACUUM, BC_PERIODIC])
@pytest.mark.parametrize("order", [1, 3, 5])
def test_rows_of_absolute_is_the_magnitude_product(order, bc):
    # |A| |x| where |A| holds sigma_t + |g|^l sigma_s on the diagonal (the two
    # parts of the diagonal taken in magnitude) and |c| / h off it: the
    # assembled matrix of albedo -> -albedo, g -> |g| in magnitude (grids of
    # >= 3 cells, so no two terms of a row share a column).
    m = _medium(order, (3, 4, 3), bc, seed=5)
    Mag, lay = assemble(order, m.dims, m.sigma_t, -m.albedo, abs(m.g), m.sigma_t_min, bc=bc)
    Mag = abs(Mag)
    x = np.random.default_rng(3).normal(size=lay.n)
    got = rows_of(order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, x, np.arange(lay.n), bc=bc,
                  absolute=True)
    np.testing.assert_allclose(got, Mag @ np.abs(x), rtol=1e-13)


def test_rows_of_absolute_bounds_neumann_rows():
    # Under Neumann two terms of a boundary row fall on one column and cancel
    # in the matrix; the term-by-term magnitude is still an upper bound.
    order, bc = 3, BC_NEUMANN
    m = _medium(order, (3, 3, 4), bc, seed=6)
    Mag, lay = assemble(order, m.dims, m.sigma_t, -m.albedo, abs(m.g), m.sigma_t_min, bc=bc)
    x = np.random.default_rng(4).normal(size=lay.n)
    got = rows_of(order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, x, np.arange(lay.n), bc=bc,
                  absolute=True)
    assert np.all(got >= abs(Mag) @ np.abs(x) * (1 - 1e-13))


def test_rows_of_with_cell_size():
    order, dims, h = 3, (4, 4, 3), 0.37
    m = _medium(order, dims, BC_VACUUM, seed=7)
    A, lay = assemble(order, dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, h=h)
    x = np.random.default_rng(5).normal(size=lay.n)
    got = rows_of(order, dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, x, np.arange(lay.n), h=h)
    np.testing.assert_allclose(got, A @ x, rtol=1e-13, atol=1e-11)


# -------------------------------------------------------- consistency -----
@pytest.mark.parametrize("bc", BCS[2:])
@pytest.mark.parametrize("order", [1, 2, 3, 5])
def test_neumann_and_mixed_row_loop_vectorised_matrix_free(order, bc):
    m = _medium(order, (3, 4, 3), bc, seed=order)
    A, lay = assemble(order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc)
    A2, _ = assemble_rows(order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc)
    assert abs(A - A2).max() < 1e-13
    op = Operator(order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc)
    x = np.random.default_rng(1).normal(size=lay.n)
    np.testing.assert_allclose(op.matvec(x), A @ x, atol=1e-12)
    np.testing.assert_allclose(op.rmatvec(x), A.T @ x, atol=1e-12)


def test_neumann_extents_include_boundary_faces():
    lay = Layout(3, (5, 4, 3), BC_NEUMANN)
    lv = Layout(3, (5, 4, 3), BC_VACUUM)
    assert lay.ext == lv.ext and lay.n == lv.n
    mixed = Layout(3, (5, 4, 1), (BC_VACUUM, BC_VACUUM, BC_PERIODIC))
    for k in range(mixed.ncoeff):
        assert mixed.ext[k][2] == 1 and mixed.ext[k][:2] == lv.ext[k][:2]


# ------------------------------------------------------ Neumann pins ------
@pytest.mark.parametrize("order", [1, 3, 5])
def test_neumann_uniform_medium_closed_form(order):
    # Uniform sigma_t, albedo and isotropic Q under Neumann on every axis:
    # L00 = Q / sigma_a everywhere and every other coefficient 0.  (The same
    # medium under the vacuum boundary leaks and does not give this.)
    n, st, alb, q = 4, 5.0, 0.8, 2.0
    shp = (n, n, n)
    st32, alb32 = np.float32(st), np.float32(alb)
    A, lay = assemble(order, (n, n, n), np.full(shp, st32), np.full(shp, alb32), 0.4, 0.0, bc=BC_NEUMANN)
    u = direct(A, rhs_isotropic(lay, np.full(shp, q)))
    sa = float(st32) * (1.0 - float(alb32))
    np.testing.assert_allclose(lay.view(u, 0), q / sa, rtol=1e-12)
    assert np.abs(u[lay.offset[1]:]).max() < 1e-12
    Av, _ = assemble(order, (n, n, n), np.full(shp, st32), np.full(shp, alb32), 0.4, 0.0, bc=BC_VACUUM)
    uv = direct(Av, rhs_isotropic(lay, np.full(shp, q)))
    assert lay.view(uv, 0).min() < 0.9 * q / sa


def _mirror(a, axes):
    """Field on (nz, ny, nx) cells -> the field on the doubled grid along the
    given axes (0 = x, 1 = y, 2 = z), reflected about the far boundary."""
    for d in axes:
        ax = 2 - d
        a = np.concatenate([a, np.flip(a, axis=ax)], axis=ax)
    return a


@pytest.mark.parametrize("axes", [(0,), (2,), (0, 1, 2)])
@pytest.mark.parametrize("order", [1, 3])
def test_neumann_boundary_is_a_mirror(order, axes):
    dims = (3, 4, 3)
    rng = np.random.default_rng(17)
    shp = (dims[2], dims[1], dims[0])
    st = rng.uniform(1.0, 10.0, size=shp).astype(np.float32)
    alb = rng.uniform(0.3, 0.9, size=shp).astype(np.float32)
    q = rng.uniform(0.0, 1.0, size=shp).astype(np.float32)
    g = 0.3
    bc_n = tuple(BC_NEUMANN if d in axes else BC_VACUUM for d in range(3))
    bc_p = tuple(BC_PERIODIC if d in axes else BC_VACUUM for d in range(3))
    dims2 = tuple(2 * dims[d] if d in axes else dims[d] for d in range(3))
    h = 1.0 / dims[0]  # same cell size on both grids
    A2, lay2 = assemble(order, dims2, _mirror(st, axes), _mirror(alb, axes), g, 0.0, bc=bc_p, h=h)
    u2 = direct(A2, rhs_isotropic(lay2, _mirror(q, axes)))
    A, lay = assemble(order, dims, st, alb, g, 0.0, bc=bc_n, h=h)
    u = direct(A, rhs_isotropic(lay, q))
    for k in range(lay.ncoeff):
        v, v2 = lay.view(u, k), lay2.view(u2, k)
        ext = lay.ext[k]
        # first half of the doubled grid; the Neumann grid's extra boundary
        # faces (index n along a mirrored axis) sit on the far mirror plane
        sl = tuple(slice(0, min(ext[2 - a], v2.shape[a])) for a in range(3))
        part = v2[sl]
        mine = v[tuple(slice(0, s) for s in part.shape)]
        np.testing.assert_allclose(mine, part, atol=1e-12)
        for d in axes:  # face classes on a mirror plane vanish
            if lay.cls[k][d] == 1:
                ax = 2 - d
                np.testing.assert_allclose(np.take(v, [0, ext[d] - 1], axis=ax), 0.0, atol=1e-12)


# ---------------------------------------------------- per-axis, 2D, h -----
@pytest.mark.parametrize("order", [1, 3, 5])
def test_two_dimensional_problem_is_one_periodic_z_cell(order):
    # A z-invariant problem with vacuum in x, y: one z-periodic cell gives the
    # same coefficients as every plane of a 3-cell z-periodic grid, and the
    # z-odd coefficients (l + |m| odd) vanish (section "2D checkerboard").
    rng = np.random.default_rng(order)
    nx, ny = 5, 4
    st2 = rng.uniform(1, 10, size=(ny, nx)).astype(np.float32)
    q2 = rng.uniform(0, 1, size=(ny, nx)).astype(np.float32)
    alb = 0.7
    bc = (BC_VACUUM, BC_VACUUM, BC_PERIODIC)
    A1, l1 = assemble(order, (nx, ny, 1), st2[None], np.full((1, ny, nx), alb, np.float32), 0.3, 0.0, bc=bc)
    u1 = direct(A1, rhs_isotropic(l1, q2[None]))
    st3 = np.repeat(st2[None], 3, axis=0)
    A3, l3 = assemble(order, (nx, ny, 3), st3, np.full(st3.shape, alb, np.float32), 0.3, 0.0, bc=bc, h=1.0 / nx)
    u3 = direct(A3, rhs_isotropic(l3, np.repeat(q2[None], 3, axis=0)))
    for k in range(l1.ncoeff):
        for z in range(3):
            np.testing.assert_allclose(l1.view(u1, k)[0], l3.view(u3, k)[z], atol=1e-12)
        l, m = sh.coeff_lm(k)
        if (l + abs(m)) % 2 == 1:
            assert np.abs(l1.view(u1, k)).max() < 1e-12
    assert np.abs(l1.view(u1, 0)).max() > 1e-3


@pytest.mark.parametrize("h", [0.05, 0.3])
def test_periodic_fourier_mode_with_cell_size(h):
    # As the Fourier-mode pin, on a domain of n*h per axis for h != 1/n.
    order = 3
    dims = (6, 4, 4)
    L = [n * h for n in dims]
    kappa = np.array([2 * pi / L[0], 2 * pi * 2 / L[1], 2 * pi / L[2]])
    st32, alb32, g = np.float32(3.0), np.float32(0.6), float(np.float32(0.35))
    shp = (dims[2], dims[1], dims[0])
    A, lay = assemble(order, dims, np.full(shp, st32), np.full(shp, alb32), g, 0.0, bc=1, h=h)
    z, y, x = np.meshgrid(*[(np.arange(n) + 0.5) * h for n in dims[::-1]], indexing="ij")
    u = direct(A, rhs_isotropic(lay, np.cos(kappa[0] * x + kappa[1] * y + kappa[2] * z)))
    T = transport_couplings(order)
    Ms = sum((2j * np.sin(kappa[d] * h / 2) / h) * T[d] for d in range(3))
    ssv = float(st32) * float(alb32)
    Ms = Ms + np.diag([float(st32) - ssv * g ** sh.coeff_lm(k)[0] for k in range(lay.ncoeff)])
    e0 = np.zeros(lay.ncoeff, dtype=complex)
    e0[0] = 1.0
    uh = np.linalg.solve(Ms, e0)
    for k in range(lay.ncoeff):
        px, py, pz = lay.positions(k)
        want = np.real(uh[k] * np.exp(1j * (kappa[0] * px * h + kappa[1] * py * h + kappa[2] * pz * h)))
        np.testing.assert_allclose(lay.view(u, k), want, atol=1e-12)
