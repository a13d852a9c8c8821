"""Pins of the C/OpenMP oracle (oracle/pn_ref.c via oracle/ref.py): its
matrix-free A and A^T equal the assembled SciPy matrix entry by entry on
small grids for every order, boundary type (vacuum, periodic, Neumann,
mixed per axis), ragged extents and an explicit cell size; its CGLS reaches
the SuperLU solution, with a carried residual that never increases (CGLS
minimises ||Q - A u|| over growing Krylov spaces)."""
import numpy as np
import pytest

from oracle.assemble import assemble, rhs_isotropic
from oracle.ref import CRef
from oracle.solve import direct
from synth import config_small


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("bc", [0, 1, 2, (1, 0, 2), (2, 2, 1)])
def test_c_operator_equals_assembled_matrix(order, bc):
    dims = (4, 3, 5) if order > 4 else (5, 4, 3)
    m = config_small(order, dims, seed=order)
    h = 0.37 if order % 2 else None
    A, lay = assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc, h=h)
    R = CRef(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc, h=h, threads=2)
    assert R.n == lay.n
    x = np.random.default_rng(order).normal(size=lay.n)
    scale = abs(A) @ np.abs(x)
    assert np.all(np.abs(R.matvec(x) - A @ x) <= 1e-13 * scale + 1e-300)
    scale_t = abs(A.T) @ np.abs(x)
    assert np.all(np.abs(R.rmatvec(x) - A.T @ x) <= 1e-13 * scale_t + 1e-300)


@pytest.mark.parametrize("order,bc", [(1, 0), (3, 0), (3, 2), (5, 1)])
def test_c_cgls_reaches_direct_solution(order, bc):
    m = config_small(order, (6, 5, 4), seed=10 + order, sigma_range=(2.0, 20.0), albedo_range=(0.5, 0.95),
                     sigma_t_min=1.0)
    A, lay = assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc)
    b = rhs_isotropic(lay, m.q00[0])
    u = direct(A, b)
    R = CRef(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc, threads=3)
    x, info = R.cgls(b, tol=1e-12)
    assert info["carried_rel_residual"] <= 1e-12
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-11
    assert np.linalg.norm(x - u) / np.linalg.norm(u) <= 1e-9
    h = info["history"]
    assert h[0] == 1.0 and np.all(np.diff(h) <= 1e-14)
    assert info["threads"] == 3


def test_c_cgls_zero_rhs():
    m = config_small(3, (3, 3, 3), seed=1)
    R = CRef(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, threads=1)
    x, info = R.cgls(np.zeros(R.n), tol=1e-10)
    assert info["iters"] == 0 and np.all(x == 0)
