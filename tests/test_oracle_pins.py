"""Pins of the FP64 oracle against what the paper and the mathematics fix
(closed forms, invariants, brute force, library routines).  CPU only."""
from math import pi, sqrt

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.special

from oracle import sh
from oracle.assemble import assemble, assemble_rows, rhs_isotropic
from oracle.apply import Operator
from oracle.closed_form import a_, b_, c_, d_, e_, f_, closed_form_table
from oracle.couplings import (coupling_list, gram_matrix, hg_phase, scattering_factors,
                              transport_couplings)
from oracle.medium import interpolate_to_class
from oracle.solve import cgls, direct
from oracle.stagger import BC_PERIODIC, BC_VACUUM, Layout, coeff_class
from synth import config_small, config_uniform_periodic, config_p1_homogeneous

ORDERS = (1, 3, 5, 7)


# ---------------------------------------------------------------- basis -----
@pytest.mark.parametrize("l", range(0, 8))
def test_assoc_legendre_matches_scipy_without_cs_phase(l):
    # scipy's lpmv includes the Condon-Shortley phase (-1)^m; the appendix's P does not.
    x = np.linspace(-0.999, 0.999, 37)
    for m in range(0, l + 1):
        ref = ((-1.0) ** m) * scipy.special.lpmv(m, l, x)
        np.testing.assert_allclose(sh.assoc_legendre(l, m, x), ref, rtol=1e-12, atol=1e-12)


def test_real_basis_is_real_and_matches_composed_form():
    rng = np.random.default_rng(0)
    th = np.arccos(rng.uniform(-1, 1, 200))
    ph = rng.uniform(0, 2 * pi, 200)
    for l in range(6):
        for m in range(-l, l + 1):
            y = sh.real_basis_from_complex(l, m, th, ph)
            assert np.abs(y.imag).max() < 1e-13
            mu = abs(m)
            base = sh.norm_K(l, mu) * sh.assoc_legendre(l, mu, np.cos(th))
            want = base if m == 0 else sqrt(2.0) * base * (np.sin(mu * ph) if m < 0 else np.cos(mu * ph))
            np.testing.assert_allclose(y.real, want, atol=1e-13)


def test_main_text_minus_form_is_not_real():
    # Reading Z1: the main-text m>0 combination with "-" is imaginary for odd m.
    th, ph = np.array([0.7]), np.array([0.3])
    bad = (1 / sqrt(2)) * (sh.complex_sh(2, -1, th, ph) - (-1.0) ** 1 * sh.complex_sh(2, 1, th, ph))
    assert abs(bad.imag[0]) > 0.1


@pytest.mark.parametrize("order", ORDERS)
def test_gram_is_identity(order):
    G = gram_matrix(order)
    np.testing.assert_allclose(G, np.eye(G.shape[0]), atol=1e-13)


def test_y00_and_l1_closed_forms():
    th = np.array([0.3, 1.1, 2.5])
    ph = np.array([0.2, 4.0, 5.5])
    k = sqrt(3.0 / (4 * pi))
    np.testing.assert_allclose(sh.real_sh(0, 0, th, ph), 1 / sqrt(4 * pi))
    np.testing.assert_allclose(sh.real_sh(1, 1, th, ph), k * np.sin(th) * np.cos(ph))
    np.testing.assert_allclose(sh.real_sh(1, -1, th, ph), k * np.sin(th) * np.sin(ph))
    np.testing.assert_allclose(sh.real_sh(1, 0, th, ph), k * np.cos(th))


# ------------------------------------------------------------ couplings -----
@pytest.mark.parametrize("order", ORDERS + (2, 4, 6))
def test_quadrature_couplings_equal_corrected_closed_form(order):
    A = transport_couplings(order)
    cf = closed_form_table(order)
    quad = {(k, d, kp): A[d, k, kp] for d in range(3) for k in range(A.shape[1])
            for kp in range(A.shape[1]) if A[d, k, kp] != 0.0}
    assert set(quad) == set(cf)
    for key, v in quad.items():
        assert abs(v - cf[key]) < 1e-13, key


def test_printed_signs_differ_exactly_on_xy():
    A = transport_couplings(5)
    cf = closed_form_table(5, printed_signs=True)
    for (k, d, kp), v in cf.items():
        want = -A[d, k, kp] if d < 2 else A[d, k, kp]
        assert abs(v - want) < 1e-13


@pytest.mark.parametrize("order,count", [(1, 6), (3, 70), (5, 214), (7, 438)])
def test_coupling_counts_and_structure(order, count):
    A = transport_couplings(order)
    cl = coupling_list(order)
    assert len(cl) == count
    assert np.abs(A - A.transpose(0, 2, 1)).max() < 1e-15
    for (k, d, kp, _) in cl:
        lk, lkp = sh.coeff_lm(k)[0], sh.coeff_lm(kp)[0]
        assert abs(lk - lkp) == 1
        pk, pkp = coeff_class(*sh.coeff_lm(k)), coeff_class(*sh.coeff_lm(kp))
        diff = [a != b for a, b in zip(pk, pkp)]
        assert diff.count(True) == 1 and diff[d]


def test_az_10_00_value():
    A = transport_couplings(1)
    assert abs(A[2, sh.coeff_index(1, 0), 0] - 1 / sqrt(3)) < 1e-15
    assert abs(A[0, sh.coeff_index(1, 1), 0] - 1 / sqrt(3)) < 1e-15
    assert abs(A[1, sh.coeff_index(1, -1), 0] - 1 / sqrt(3)) < 1e-15


def test_coefficient_identities():
    for l in range(0, 7):
        for m in range(-l, l + 1):
            assert abs(a_(l, m) - a_(l, -m)) < 1e-15
            if l >= 1 and abs(m) < l:
                assert abs(b_(l, m) - b_(l, -m)) < 1e-15
            if l + m + 1 >= 0 and l - m + 1 >= 0:
                assert abs(c_(l, m) - e_(l, -m)) < 1e-15
            if l >= 1 and (l - m) * (l - m - 1) >= 0 and (l + m) * (l + m - 1) >= 0:
                assert abs(d_(l, m) - f_(l, -m)) < 1e-15


@pytest.mark.parametrize("g", [0.0, 0.3, 0.5, -0.4])
def test_hg_scattering_factor_is_g_power_l(g):
    f = scattering_factors(7, lambda mu: hg_phase(g, mu))
    np.testing.assert_allclose(f, [g ** l for l in range(8)], atol=1e-12)


# ------------------------------------------------------ layout / medium -----
def test_unknown_counts():
    assert Layout(1, (16, 16, 16)).n == 17152
    assert Layout(3, (64, 64, 64)).n == 4268417
    assert Layout(3, (96, 96, 96)).n == 14322241
    assert Layout(5, (128, 128, 128)).n == 76237059
    assert Layout(7, (96, 96, 96)).n == 57400710


def test_class_sizes_p5():
    lay = Layout(5, (4, 4, 4))
    from collections import Counter
    c = Counter(lay.cls)
    assert c[(0, 0, 0)] == 6 and c[(1, 0, 0)] == 6 and c[(0, 1, 0)] == 6 and c[(0, 0, 1)] == 6
    assert c[(1, 1, 0)] == 3 and c[(1, 0, 1)] == 3 and c[(0, 1, 1)] == 3 and c[(1, 1, 1)] == 3


def test_interpolation_brute_force():
    f = np.array([[[1.0, 3.0]]])          # nz=1, ny=1, nx=2
    np.testing.assert_allclose(interpolate_to_class(f, (1, 0, 0), (3, 1, 1), BC_VACUUM)[0, 0], [1, 2, 3])
    np.testing.assert_allclose(interpolate_to_class(f, (1, 0, 0), (2, 1, 1), BC_PERIODIC)[0, 0], [2, 2])
    np.testing.assert_allclose(interpolate_to_class(f, (0, 0, 0), (2, 1, 1), BC_VACUUM)[0, 0], [1, 3])
    g = np.arange(8.0).reshape(2, 2, 2)   # value = 4z + 2y + x
    c = interpolate_to_class(g, (1, 1, 1), (3, 3, 3), BC_VACUUM)
    assert c[1, 1, 1] == pytest.approx(3.5)       # interior corner: mean of all 8
    assert c[0, 0, 0] == pytest.approx(0.0)       # clamped: cell (0,0,0) only
    assert c[2, 0, 1] == pytest.approx(4.5)       # z clamped to cell 1, y cell 0, x mean of 0,1


# ------------------------------------------------------------- assembly -----
@pytest.mark.parametrize("bc", [BC_VACUUM, BC_PERIODIC])
@pytest.mark.parametrize("order", [1, 3, 5])
def test_vectorised_assembly_and_matrix_free_match_row_loop(order, bc):
    m = config_small(order, (3, 4, 2), seed=order, bc=bc)
    A, lay = assemble(order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc)
    A2, _ = assemble_rows(order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc)
    assert abs(A - A2).max() < 1e-13
    op = Operator(order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc)
    x = np.random.default_rng(1).normal(size=lay.n)
    np.testing.assert_allclose(op.matvec(x), A @ x, atol=1e-12)
    np.testing.assert_allclose(op.rmatvec(x), A.T @ x, atol=1e-12)


def test_p1_single_cell_by_hand():
    st, alb, g = 4.0, 0.75, float(np.float32(0.2))
    shp = (1, 1, 1)
    A, lay = assemble(1, (1, 1, 1), np.full(shp, st), np.full(shp, alb), g, 0.0)
    c = 1 / sqrt(3)
    sa, d1 = st - alb * st, st - g * alb * st
    # layout order: L00 | L1-1 (y faces 0,1) | L10 (z faces 0,1) | L11 (x faces 0,1)
    M = np.array([[sa, -c, c, -c, c, -c, c],
                  [c, d1, 0, 0, 0, 0, 0],
                  [-c, 0, d1, 0, 0, 0, 0],
                  [c, 0, 0, d1, 0, 0, 0],
                  [-c, 0, 0, 0, d1, 0, 0],
                  [c, 0, 0, 0, 0, d1, 0],
                  [-c, 0, 0, 0, 0, 0, d1]])
    np.testing.assert_allclose(A.toarray(), M, atol=1e-15)


@pytest.mark.parametrize("order", [1, 3, 5])
@pytest.mark.parametrize("bc", [BC_VACUUM, BC_PERIODIC])
def test_transport_part_is_skew(order, bc):
    # x^T A x = sum_k diag_k x_k^2 for every x, and y^T (A x) = x^T (A^T y).
    m = config_small(order, (4, 3, 5), seed=11, bc=bc)
    op = Operator(order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc)
    rng = np.random.default_rng(5)
    x, y = rng.normal(size=op.n), rng.normal(size=op.n)
    lay = op.layout
    quad = sum(float(np.sum(op.diag[k] * lay.view(x, k) ** 2)) for k in range(lay.ncoeff))
    assert abs(x @ op.matvec(x) - quad) < 1e-9 * abs(quad)
    assert abs(y @ op.matvec(x) - x @ op.rmatvec(y)) < 1e-9 * np.linalg.norm(x) * np.linalg.norm(y) * 100


# ------------------------------------------------------- closed-form solves -
@pytest.mark.parametrize("order", [1, 3, 5])
def test_uniform_periodic_isotropic(order):
    m = config_uniform_periodic(n=4, order=order, sigma_t=5.0, albedo=0.8, g=0.4, q=2.0)
    A, lay = assemble(order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=1)
    u = direct(A, rhs_isotropic(lay, m.q00[0]))
    sa = float(np.float32(5.0)) * (1 - float(np.float32(0.8)))
    np.testing.assert_allclose(lay.view(u, 0), 2.0 / sa, rtol=1e-12)
    assert np.abs(u[lay.offset[1]:]).max() < 1e-12


def test_uniform_periodic_anisotropic_source():
    order, g = 3, 0.4
    m = config_uniform_periodic(n=3, order=order, sigma_t=5.0, albedo=0.8, g=g)
    A, lay = assemble(order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=1)
    st, ss = float(np.float32(5.0)), float(np.float32(5.0)) * float(np.float32(0.8))
    g = float(np.float32(g))
    q = np.arange(1.0, lay.ncoeff + 1)
    b = np.zeros(lay.n)
    for k in range(lay.ncoeff):
        lay.view(b, k)[...] = q[k]
    u = direct(A, b)
    for k in range(lay.ncoeff):
        l = sh.coeff_lm(k)[0]
        np.testing.assert_allclose(lay.view(u, k), q[k] / (st - ss * g ** l), rtol=1e-12)


@pytest.mark.parametrize("order", [1, 3, 5])
def test_periodic_fourier_mode(order):
    dims = (8, 6, 4)
    h = 1.0 / dims[0]
    kappa = np.array([2 * pi * 1 / (dims[0] * h), 2 * pi * 2 / (dims[1] * h), 2 * pi * 1 / (dims[2] * h)])
    st, alb, g = 3.0, 0.6, float(np.float32(0.35))
    shp = (dims[2], dims[1], dims[0])
    st32, alb32 = np.float32(st), np.float32(alb)
    A, lay = assemble(order, dims, np.full(shp, st32), np.full(shp, alb32), g, 0.0, bc=1)
    z, y, x = np.meshgrid(*[(np.arange(n) + 0.5) * h for n in dims[::-1]], indexing="ij")
    b = rhs_isotropic(lay, np.cos(kappa[0] * x + kappa[1] * y + kappa[2] * z))
    u = direct(A, b)
    # per-mode dense system from the couplings (independent of the sparse indexing)
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


@pytest.mark.parametrize("order", [1, 3])
def test_second_order_convergence_to_the_continuous_solution(order):
    # The continuous P_N system for a periodic homogeneous medium and a single
    # Fourier-mode source has the exact solution Re(u e^{i kappa.x}) with
    # (sum_d i kappa_d A_d + diag(sigma_t - g^l sigma_s)) u = e_0 (derivatives
    # of the continuous equations, not the staggered differences).  The
    # discrete solution sampled at each coefficient's staggered positions must
    # approach it at second order in h ("Precomputation": central differences
    # on the staggered grid).
    st, alb, g = 4.0, 0.7, float(np.float32(0.3))
    st32, alb32 = np.float32(st), np.float32(alb)
    T = transport_couplings(order)
    errs = []
    for n in (8, 16, 32):
        # kappa_z = 0: the solution is z-invariant, two periodic cells in z carry it exactly
        dims = (n, n, 2)
        h = 1.0 / n
        kappa = 2 * pi * np.array([1.0, 1.0, 0.0])
        shp = (2, n, n)
        A, lay = assemble(order, dims, np.full(shp, st32), np.full(shp, alb32), g, 0.0, bc=1)
        z, y, x = np.meshgrid(*[(np.arange(m) + 0.5) * h for m in dims[::-1]], indexing="ij")
        u = direct(A, rhs_isotropic(lay, np.cos(kappa[0] * x + kappa[1] * y + kappa[2] * z)))
        M = sum(1j * kappa[d] * T[d] for d in range(3))
        ssv = float(st32) * float(alb32)
        M = M + np.diag([float(st32) - ssv * g ** sh.coeff_lm(k)[0] for k in range(lay.ncoeff)])
        e0 = np.zeros(lay.ncoeff, dtype=complex)
        e0[0] = 1.0
        uc = np.linalg.solve(M, e0)
        err = 0.0
        for k in range(lay.ncoeff):
            px, py, pz = lay.positions(k)
            want = np.real(uc[k] * np.exp(1j * (kappa[0] * px * h + kappa[1] * py * h + kappa[2] * pz * h)))
            err = max(err, float(np.abs(lay.view(u, k) - want).max()))
        errs.append(err)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.6 and 3.7 < r2 < 4.3, (errs, r1, r2)


def test_periodic_heterogeneous_balance():
    m = config_small(3, (5, 4, 3), seed=2, bc=1)
    A, lay = assemble(3, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=1)
    u = direct(A, rhs_isotropic(lay, m.q00[0]))
    st = np.maximum(m.sigma_t.astype(np.float64), m.sigma_t_min)
    sa = st - m.albedo.astype(np.float64) * st
    assert abs(np.sum(sa * lay.view(u, 0)) - np.sum(m.q00[0].astype(np.float64))) < 1e-10 * np.sum(m.q00[0])


def test_2d_reduction_z_invariant():
    order = 5
    dims = (6, 5, 3)
    rng = np.random.default_rng(4)
    st2 = rng.uniform(1, 10, size=(5, 6))
    q2 = rng.uniform(0, 1, size=(5, 6))
    st = np.repeat(st2[None], 3, axis=0).astype(np.float32)
    q = np.repeat(q2[None], 3, axis=0).astype(np.float32)
    A, lay = assemble(order, dims, st, np.full(st.shape, 0.7, np.float32), 0.3, 0.0, bc=1)
    u = direct(A, rhs_isotropic(lay, q))
    zodd = [k for k in range(lay.ncoeff) if lay.cls[k][2] == 1]
    assert len(zodd) > 0
    for k in zodd:
        assert np.abs(lay.view(u, k)).max() < 1e-12
    assert np.abs(lay.view(u, 0)).max() > 1e-3


def test_mirror_symmetry_x():
    order = 3
    dims = (6, 4, 4)
    rng = np.random.default_rng(9)
    st = rng.uniform(1, 10, size=(4, 4, 3))
    st = np.concatenate([st, st[:, :, ::-1]], axis=2).astype(np.float32)
    q = rng.uniform(0, 1, size=(4, 4, 3))
    q = np.concatenate([q, q[:, :, ::-1]], axis=2).astype(np.float32)
    A, lay = assemble(order, dims, st, np.full(st.shape, 0.8, np.float32), 0.2, 0.0)
    u = direct(A, rhs_isotropic(lay, q))
    for k in range(lay.ncoeff):
        v = lay.view(u, k)
        sign = -1.0 if lay.cls[k][0] == 1 else 1.0
        np.testing.assert_allclose(v, sign * v[:, :, ::-1], atol=1e-12)


def test_p1_schur_complement_is_diffusion():
    # Eliminating the face unknowns of P1 leaves sigma_a u - div(1/(3 s') grad u) = Q
    # on the cell centres with s' = sigma_t - g sigma_s at the faces (P1 = CDA).
    dims = (3, 3, 3)
    m = config_small(1, dims, seed=3, g=0.25)
    A, lay = assemble(1, dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min)
    D = A.toarray()
    nc = lay.size[0]
    Acc, Acf, Afc, Aff = D[:nc, :nc], D[:nc, nc:], D[nc:, :nc], D[nc:, nc:]
    S = Acc - Acf @ np.linalg.solve(Aff, Afc)
    h = 1.0 / 3
    st = np.maximum(m.sigma_t.astype(np.float64), m.sigma_t_min)
    ss = m.albedo.astype(np.float64) * st
    sp_ = st - float(np.float32(m.g)) * ss
    n = 3
    W = np.zeros((nc, nc))
    idx = lambda x, y, z: (z * n + y) * n + x
    for z in range(n):
        for y in range(n):
            for x in range(n):
                i = idx(x, y, z)
                W[i, i] += st[z, y, x] - ss[z, y, x]
                for d in range(3):
                    for s in (-1, 1):
                        c = [x, y, z]
                        nb = list(c)
                        nb[d] += s
                        # face value: mean of the two cells (clamped at the boundary)
                        cl = [min(max(v, 0), n - 1) for v in nb]
                        sf = 0.5 * (sp_[z, y, x] + sp_[cl[2], cl[1], cl[0]])
                        coef = 1.0 / (3.0 * sf * h * h)
                        W[i, i] += coef
                        if 0 <= nb[d] < n:
                            W[i, idx(*nb)] -= coef
    np.testing.assert_allclose(S, W, atol=1e-10)


# ------------------------------------------------------------------ solve ---
def test_direct_residual_and_cgls_agreement():
    m = config_small(3, (5, 4, 6), seed=8)
    A, lay = assemble(3, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min)
    b = rhs_isotropic(lay, m.q00[0])
    u = direct(A, b)
    assert np.linalg.norm(b - A @ u) / np.linalg.norm(b) < 1e-12
    x, info = cgls(lambda v: A @ v, lambda v: A.T @ v, b, tol=1e-13)
    assert info["rel_residual"] < 1e-12
    assert np.linalg.norm(x - u) / np.linalg.norm(u) < 1e-10


def test_config_p1_direct_residual():
    m = config_p1_homogeneous()
    A, lay = assemble(1, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min)
    b = rhs_isotropic(lay, m.q00[0])
    u = direct(A, b)
    assert np.linalg.norm(b - A @ u) / np.linalg.norm(b) < 1e-12
    # symmetric source, symmetric medium: L00 is symmetric in x
    v = lay.view(u, 0)
    np.testing.assert_allclose(v, v[:, :, ::-1], rtol=1e-10)


@pytest.mark.parametrize("order", [1, 2, 3, 5, 7])
@pytest.mark.parametrize("bc", [0, 1, (0, 1, 0)])
def test_even_odd_block_structure(order, bc):
    # The transport couples bands l and l +- 1 only, and a coefficient's band
    # parity equals the parity of its staggering class, so with the unknowns
    # split by band parity A = [[D_e, T_eo], [T_oe, D_o]] with D_e, D_o
    # diagonal and, the transport being skew (vacuum / periodic), T_oe =
    # -T_eo^T: the even-parity Schur complement S = D_e - T_eo D_o^-1 T_oe
    # is symmetric positive definite (the GPU's even-parity solver relies on
    # all of it).
    from oracle.sh import coeff_lm
    from oracle.stagger import class_of_k
    m = config_small(order, (4, 3, 5) if order < 5 else (3, 2, 3), seed=order)
    A, lay = assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc)
    for k in range(lay.ncoeff):
        assert coeff_lm(k)[0] % 2 == sum(class_of_k(k)) % 2
    par = np.concatenate([np.full(lay.size[k], coeff_lm(k)[0] % 2) for k in range(lay.ncoeff)])
    E, O = np.nonzero(par == 0)[0], np.nonzero(par == 1)[0]
    A = A.tocsr()
    Aee, Aoo = A[E][:, E], A[O][:, O]
    assert abs(Aee - sp.diags(Aee.diagonal())).max() == 0 and abs(Aoo - sp.diags(Aoo.diagonal())).max() == 0
    Aeo, Aoe = A[E][:, O], A[O][:, E]
    assert abs(Aoe + Aeo.T).max() <= 1e-12 * abs(Aeo).max()
    S = (sp.diags(Aee.diagonal()) - Aeo @ sp.diags(1.0 / Aoo.diagonal()) @ Aoe).toarray()
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    assert np.linalg.eigvalsh(0.5 * (S + S.T)).min() > 0
    # and the Schur solve plus back-substitution is the solution of A u = Q
    b = rhs_isotropic(lay, m.q00[0])
    de, do = Aee.diagonal(), Aoo.diagonal()
    ue = np.linalg.solve(S, b[E] - Aeo @ (b[O] / do))
    u = np.zeros(lay.n)
    u[E] = ue
    u[O] = (b[O] - Aoe @ ue) / do
    assert np.linalg.norm(A @ u - b) <= 1e-10 * np.linalg.norm(b)


def test_neumann_breaks_the_skew_coupling():
    # under the Neumann boundary the redirected entries make T_oe != -T_eo^T
    from oracle.sh import coeff_lm
    m = config_small(3, (4, 3, 5), seed=9)
    A, lay = assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=2)
    par = np.concatenate([np.full(lay.size[k], coeff_lm(k)[0] % 2) for k in range(lay.ncoeff)])
    E, O = np.nonzero(par == 0)[0], np.nonzero(par == 1)[0]
    A = A.tocsr()
    assert abs(A[O][:, E] + A[E][:, O].T).max() > 1.0
