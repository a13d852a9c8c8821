"""Pins of the diffusion oracle (oracle/cda.py) and of the validation
workloads of section "Results" (CPU only).

* The CDA operator equals the Schur complement that the assembled staggered
  P_1 matrix leaves on the cell centres once its face unknowns are eliminated,
  for every boundary type, per-axis boundaries, g != 0 and h != 1/n: this
  pins it to the P_N assembly, which is pinned to quadrature elsewhere, and is
  the paper's statement that P_1 equals CDA.
* It is symmetric positive definite; a uniform periodic medium with uniform
  emission gives phi = Q / sigma_a; its conjugate-gradient path agrees with
  SuperLU.
* The checkerboard workload has the lattice geometry (12 absorbing blocks,
  the source block in the centre) and, being z-invariant, its P_N solution
  has vanishing l + |m| odd coefficients; the point-source workload is
  mirror-symmetric, so its P_N solution is too (the parity of each
  coefficient under the reflection of an axis is its staggering class).
"""
import numpy as np
import pytest

from oracle.assemble import assemble, rhs_isotropic
from oracle.cda import cda_matrix, cda_solve
from oracle.sh import coeff_lm
from oracle.solve import direct
from synth import checkerboard_blocks, config_checkerboard, config_point_source, config_small

VAC, PER, NEU = 0, 1, 2


def p1_schur(m, bc, h=None):
    A, lay = assemble(1, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc, h=h)
    D = A.toarray()
    nc = lay.size[0]
    Acc, Acf, Afc, Aff = D[:nc, :nc], D[:nc, nc:], D[nc:, :nc], D[nc:, nc:]
    return Acc - Acf @ np.linalg.solve(Aff, Afc), lay


@pytest.mark.parametrize("dims,bc,h", [((4, 3, 3), VAC, None), ((4, 3, 3), NEU, None), ((4, 3, 5), PER, None),
                                       ((5, 4, 3), (VAC, PER, NEU), 0.37), ((4, 4, 1), (VAC, VAC, PER), 0.5),
                                       ((1, 1, 1), VAC, None), ((3, 2, 2), (NEU, VAC, PER), None)])
def test_cda_is_the_p1_schur_complement(dims, bc, h):
    m = config_small(1, dims, seed=5, g=0.35, sigma_range=(0.5, 12.0), albedo_range=(0.2, 0.99))
    S, lay = p1_schur(m, bc, h)
    W = cda_matrix(dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc, h=h).toarray()
    assert W.shape == S.shape
    np.testing.assert_allclose(W, S, rtol=1e-12, atol=1e-10 * np.abs(S).max())


def test_cda_symmetric_positive_definite():
    m = config_small(1, (5, 4, 3), seed=6, g=0.2)
    W = cda_matrix(m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=(VAC, NEU, PER)).toarray()
    np.testing.assert_allclose(W, W.T, rtol=0, atol=1e-12 * np.abs(W).max())
    assert np.linalg.eigvalsh(W).min() > 0


def test_cda_uniform_periodic_closed_form():
    dims = (5, 4, 3)
    st = np.full((3, 4, 5), np.float32(6.0))
    al = np.full((3, 4, 5), np.float32(0.75))
    phi = cda_solve(dims, st, al, 0.3, 0.0, np.full((3, 4, 5), 2.0), bc=PER)
    sa = float(np.float32(6.0)) * (1.0 - float(np.float32(0.75)))
    np.testing.assert_allclose(phi, 2.0 / sa, rtol=1e-12)


def test_cda_conjugate_gradients_agrees_with_direct():
    m = config_point_source(1, n=12)
    q = m.q00[0]
    a = cda_solve(m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, q)
    b = cda_solve(m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, q, direct_max=0, tol=1e-14)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-12


def test_p1_fluence_equals_cda_solution():
    # the end-to-end form of the paper's "P_1 equals CDA" on the point source
    m = config_point_source(1, n=10)
    A, lay = assemble(1, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min)
    u = direct(A, rhs_isotropic(lay, m.q00[0]))
    phi = cda_solve(m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, m.q00[0])
    np.testing.assert_allclose(lay.view(u, 0), phi, rtol=1e-11, atol=1e-14 * np.abs(phi).max())


def test_checkerboard_geometry():
    kind = checkerboard_blocks()
    assert (kind == 1).sum() == 12 and kind[3, 3] == 2 and (kind == 2).sum() == 1
    assert kind[0].sum() == 0 and kind[6].sum() == 0 and kind[:, 0].sum() == 0 and kind[:, 6].sum() == 0
    assert np.array_equal(kind, kind.T) and np.array_equal(kind, kind[::-1, ::-1])
    m = config_checkerboard(1, n=71)
    assert m.dims == (71, 71, 1) and abs(m.h - 7.0 / 71) < 1e-15 and m.bc == (0, 0, 1)
    st, al, q = m.sigma_t[0], m.albedo[0], m.q00[0][0]
    assert set(np.unique(st)) == {1.0, 10.0} and set(np.unique(al)) == {0.0, 1.0}
    assert np.all((st == 10.0) == (al == 0.0))
    # the cell (35, 35) is the centre of the source block; (15, 15) is in the absorbing block (1, 1)
    assert q[35, 35] == 1.0 and st[15, 15] == 10.0 and q.sum() == 11 * 11


@pytest.mark.parametrize("order", [2, 3])
def test_checkerboard_z_odd_coefficients_vanish(order):
    m = config_checkerboard(order, n=14)
    A, lay = assemble(order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=m.bc, h=m.h)
    u = direct(A, rhs_isotropic(lay, m.q00[0]))
    for k in range(lay.ncoeff):
        l, mm = coeff_lm(k)
        if (l + abs(mm)) % 2 == 1:
            assert np.abs(lay.view(u, k)).max() == 0.0
    assert lay.view(u, 0).min() > 0


@pytest.mark.parametrize("order", [1, 2, 3])
def test_point_source_mirror_symmetry(order):
    m = config_point_source(order, n=6)
    A, lay = assemble(order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min)
    u = direct(A, rhs_isotropic(lay, m.q00[0]))
    scale = np.abs(u).max()
    for k in range(lay.ncoeff):
        v = lay.view(u, k)
        for d, ax in ((0, 2), (1, 1), (2, 0)):
            sign = -1.0 if lay.cls[k][d] == 1 else 1.0
            np.testing.assert_allclose(v, sign * np.flip(v, axis=ax), rtol=0, atol=1e-12 * scale)
