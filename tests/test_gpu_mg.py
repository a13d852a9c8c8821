"""GPU parity of the even-parity PCG with the multigrid preconditioner
(PN_VARIANT_SCHUR_MG, AUTO on vacuum boundaries): B r = 0.6 M r + P V(P^T r),
one aggregation V-cycle per even coefficient on the Galerkin coarse
operators of the Schur complement's diagonal blocks.

The preconditioner changes only the iteration count, so every solve must
meet the FP64 residual measured by the oracle's assembled matrix and lie
within 1e-5 (rel-L2) of SuperLU -- orders 1..7, ragged, odd and degenerate
grids (one level or several), heterogeneous media; it must take fewer
iterations than the Jacobi-preconditioned form on heterogeneous media; AUTO
equals it bitwise for odd orders with at least 2^17 even-band unknowns and
the Jacobi form otherwise; periodic and mixed axes (cut at the seam in the
preconditioner only) solve to the same bar; the variant is refused with a
Neumann axis and in FP64.  The preconditioner itself matches its FP64
definition (tests/mg_reference.py, from the oracle's assembled Schur
complement) element by element on grids that take every path of its kernels
(one-block coarsest level, the one-launch tail from level 1, 2 or 3, wide
passes, a periodic seam), and stays symmetric, positive and linear at 96^3,
where the wide passes march several z planes per thread.
"""
import numpy as np
import pytest
import torch

from oracle.assemble import assemble, rhs_isotropic
from oracle.solve import direct
from synth import config_p3_fbm, config_p5_nebula, config_small

pytestmark = pytest.mark.gpu
VAC, PER, NEU = 0, 1, 2


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def auto_variant(s):
    """The inner solver AUTO picks on the register-window stencil."""
    return "schur_mg" if (s.layout.order % 2 == 1 and s.even_unknowns() >= 1 << 17) else "schur"


def solver(m, bc=VAC):
    from paper_1807_00410_amd.solver import Solver
    return Solver(m.order, m.dims, dev(m.sigma_t), dev(m.albedo), g=m.g, sigma_t_min=m.sigma_t_min, bc=bc)


# (order, dims, oracle check): SuperLU where it finishes in seconds, the
# oracle's residual of the assembled matrix on the larger (multi-level) grids
CASES = [(1, (11, 9, 8), "direct"), (2, (8, 7, 6), "direct"), (3, (10, 9, 7), "direct"), (4, (7, 6, 5), "direct"),
         (5, (8, 7, 6), "direct"), (6, (6, 5, 5), "direct"), (7, (5, 5, 4), "direct"), (3, (1, 1, 1), "direct"),
         (5, (2, 1, 3), "direct"), (3, (17, 3, 9), "direct"), (1, (33, 31, 29), "direct"), (3, (14, 12, 13), "direct"),
         (3, (24, 20, 22), "residual"), (5, (19, 21, 18), "residual"), (7, (12, 11, 13), "residual")]


@pytest.mark.parametrize("order,dims,check", CASES)
def test_mg_solve_vs_oracle(order, dims, check):
    print("case mg-solve order=%d dims=%s" % (order, dims), flush=True)
    m = config_small(order, dims, seed=90 + order, sigma_range=(1.0, 40.0), albedo_range=(0.5, 0.99),
                     sigma_t_min=1.0)
    A, lay = assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min)
    b = rhs_isotropic(lay, m.q00[0])
    s = solver(m)
    x, info = s.solve(s.rhs_from_q00(dev(m.q00[0])), tol=1e-8, variant="schur_mg")
    xs = x.cpu().numpy()
    s.close()
    res = np.linalg.norm(b - A @ xs) / np.linalg.norm(b)
    err = float("nan")
    if check == "direct":
        u = direct(A, b)
        err = np.linalg.norm(xs - u) / np.linalg.norm(u)
    print("iters %d outer %d residual %.3g error %.3g" % (info["inner_iters"], info["outer_iters"], res, err),
          flush=True)
    assert info["status"] == 0 and res <= 1.01e-8
    assert abs(res - info["rel_residual"]) <= 1e-11
    if check == "direct":
        assert err <= 1e-5


@pytest.mark.parametrize("name", ["p5_nebula_32", "p3_fbm_40"])
def test_mg_fewer_iterations_than_jacobi(name):
    print("case mg-iterations %s" % name, flush=True)
    m = config_p5_nebula(n=32, seed=3) if name == "p5_nebula_32" else config_p3_fbm(n=40, seed=1)
    s = solver(m)
    rhs = s.rhs_from_q00(dev(m.q00[0]))
    xm, im = s.solve(rhs, tol=1e-8, variant="schur_mg")
    xj, ij = s.solve(rhs, tol=1e-8, variant="schur")
    xa, ia = s.solve(rhs, tol=1e-8)
    assert auto_variant(s) == "schur_mg"
    s.close()
    print("iterations: multigrid %d, Jacobi %d" % (im["inner_iters"], ij["inner_iters"]), flush=True)
    assert im["status"] == 0 and ij["status"] == 0
    assert im["inner_iters"] * 2 <= ij["inner_iters"]
    assert ia["inner_iters"] == im["inner_iters"] and torch.equal(xa, xm)
    d = (xm - xj).norm() / xj.norm()
    assert float(d) <= 1e-6


@pytest.mark.parametrize("order,dims,bc", [(3, (8, 7, 6), PER), (5, (9, 8, 7), (VAC, VAC, PER)),
                                           (3, (12, 11, 1), (VAC, VAC, PER)), (5, (7, 9, 8), (PER, VAC, PER)),
                                           (1, (16, 14, 12), (PER, PER, VAC))])
def test_mg_periodic_axes_vs_direct(order, dims, bc):
    print("case mg-periodic order=%d dims=%s bc=%s" % (order, dims, bc), flush=True)
    m = config_small(order, dims, seed=40 + order, sigma_range=(1.0, 30.0), albedo_range=(0.5, 0.99),
                     sigma_t_min=1.0)
    A, lay = assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc)
    b = rhs_isotropic(lay, m.q00[0])
    u = direct(A, b)
    s = solver(m, bc)
    rhs = s.rhs_from_q00(dev(m.q00[0]))
    x, info = s.solve(rhs, tol=1e-8, variant="schur_mg")
    xa, ia = s.solve(rhs, tol=1e-8)
    xj, ij = s.solve(rhs, tol=1e-8, variant=auto_variant(s))
    s.close()
    xs = x.cpu().numpy()
    res = np.linalg.norm(b - A @ xs) / np.linalg.norm(b)
    err = np.linalg.norm(xs - u) / np.linalg.norm(u)
    print("iters %d residual %.3g error %.3g" % (info["inner_iters"], res, err), flush=True)
    assert info["status"] == 0 and res <= 1.01e-8 and err <= 1e-5
    assert ia["inner_iters"] == ij["inner_iters"] and torch.equal(xa, xj)


def test_mg_refused_with_neumann_and_fp64():
    from paper_1807_00410_amd.solver import PnError
    m = config_small(3, (8, 7, 6), seed=5, sigma_range=(2.0, 20.0), sigma_t_min=1.0)
    for bc in (NEU, (VAC, NEU, PER)):
        s = solver(m, bc)
        rhs = s.rhs_from_q00(dev(m.q00[0]))
        with pytest.raises(PnError):
            s.solve(rhs, tol=1e-8, variant="schur_mg")
        s.close()
    s = solver(m)
    with pytest.raises(PnError):
        s.solve(s.rhs_from_q00(dev(m.q00[0])), tol=1e-8, precision="fp64", variant="schur_mg")
    s.close()


def test_mg_repeated_solves_and_warm_start():
    # the operators are rebuilt per solve; a second solve and a warm start
    # give the same answer
    m = config_p3_fbm(n=20, seed=4)
    A, lay = assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min)
    b = rhs_isotropic(lay, m.q00[0])
    s = solver(m)
    rhs = s.rhs_from_q00(dev(m.q00[0]))
    x1, i1 = s.solve(rhs, tol=1e-8, variant="schur_mg")
    x2, i2 = s.solve(rhs, tol=1e-8, variant="schur_mg")
    assert i1["inner_iters"] == i2["inner_iters"] and torch.equal(x1, x2)
    x3, i3 = s.solve(rhs, x=x1.clone(), tol=1e-10, variant="schur_mg", use_guess=True)
    s.close()
    xs = x3.cpu().numpy()
    assert i3["status"] == 0 and np.linalg.norm(b - A @ xs) / np.linalg.norm(b) <= 1.01e-10


def test_apply_precond_definitions():
    # Jacobi: z_e = bf16(1 / diag(S)) r_e with diag(S) from the oracle's
    # matrix, z_o = 0; multigrid: B symmetric positive definite and linear
    import scipy.sparse as sp
    from oracle.sh import coeff_lm
    m = config_small(5, (9, 8, 7), seed=11, sigma_range=(1.0, 30.0), sigma_t_min=1.0)
    A, lay = assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min)
    par = np.concatenate([np.full(lay.size[k], coeff_lm(k)[0] % 2) for k in range(lay.ncoeff)])
    E, O = np.nonzero(par == 0)[0], np.nonzero(par == 1)[0]
    A = A.tocsr()
    S = sp.diags(A[E][:, E].diagonal()) - A[E][:, O] @ sp.diags(1.0 / A[O][:, O].diagonal()) @ A[O][:, E]
    dS = S.diagonal()
    s = solver(m)
    rng = np.random.default_rng(4)
    r = rng.normal(size=lay.n).astype(np.float32)
    z = s.apply_precond(dev(r), "schur").cpu().numpy().astype(np.float64)
    assert np.all(z[O] == 0.0)
    ref = r[E].astype(np.float64) / dS
    assert np.all(np.abs(z[E] - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-30)
    u = rng.normal(size=lay.n).astype(np.float32)
    v = rng.normal(size=lay.n).astype(np.float32)
    Bu = s.apply_precond(dev(u)).cpu().numpy().astype(np.float64)
    Bv = s.apply_precond(dev(v)).cpu().numpy().astype(np.float64)
    Buv = s.apply_precond(dev(u + 2.0 * v)).cpu().numpy().astype(np.float64)
    assert np.all(Bu[O] == 0.0)
    uv, vu = float(u.astype(np.float64) @ Bv), float(v.astype(np.float64) @ Bu)
    scale = float(np.abs(u) @ np.abs(Bv))
    assert abs(uv - vu) <= 1e-5 * scale
    assert float(u.astype(np.float64) @ Bu) > 0 and float(v.astype(np.float64) @ Bv) > 0
    lin = Buv - (Bu + 2.0 * Bv)
    assert np.abs(lin).max() <= 1e-5 * np.abs(Buv).max()
    from paper_1807_00410_amd.solver import PnError
    with pytest.raises(PnError):
        s.apply_precond(dev(r), 2)  # PN_VARIANT_CG has no such preconditioner
    s.close()


# (order, dims, bc): level 1 is the coarsest (one-block coarsest kernel);
# the one-launch tail from level 1; wide passes on level 1, tail from level 2;
# wide passes on levels 1-2, tail from level 3; a periodic axis (cut at the
# seam) with the tail from level 1; P7 (28 even coefficients, 28 tail blocks)
REF_CASES = [(5, (9, 8, 7), VAC), (3, (20, 18, 16), VAC), (3, (24, 20, 22), VAC), (1, (48, 44, 40), VAC),
             (3, (20, 18, 16), (VAC, PER, VAC)), (7, (12, 11, 13), VAC)]


@pytest.mark.parametrize("order,dims,bc", REF_CASES)
def test_mg_preconditioner_vs_reference(order, dims, bc):
    # B r element by element against the FP64 definition (tests/mg_reference.py)
    from mg_reference import apply_mg
    print("case mg-reference order=%d dims=%s bc=%s" % (order, dims, bc), flush=True)
    m = config_small(order, dims, seed=60 + order, sigma_range=(1.0, 30.0), albedo_range=(0.5, 0.99),
                     sigma_t_min=1.0)
    A, lay = assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=bc)
    s = solver(m, bc)
    rng = np.random.default_rng(7)
    r = rng.normal(size=lay.n).astype(np.float32)
    zj = s.apply_precond(dev(r), "schur").cpu().numpy()
    z = s.apply_precond(dev(r), "schur_mg").cpu().numpy().astype(np.float64)
    s.close()
    ref = apply_mg(A, lay, r, zj)
    err = float(np.linalg.norm(z - ref) / np.linalg.norm(ref))
    worst = float(np.abs(z - ref).max() / np.abs(ref).max())
    print("rel-L2 %.3g, largest difference %.3g of the largest entry" % (err, worst), flush=True)
    # FP32 arithmetic through at most a dozen levels: measured 6e-8 - 1.3e-7
    assert err <= 1e-6 and worst <= 1e-6


def test_mg_preconditioner_symmetric_at_96():
    # P5 on 96^3: the large-level passes march several z planes per thread
    # (level 1 holds more than 2^20 points); B stays symmetric, positive and
    # linear (properties of the definition at any size)
    print("case mg-properties P5 96^3", flush=True)
    m = config_p5_nebula(n=96, seed=3)
    s = solver(m)
    g = torch.Generator(device="cuda").manual_seed(5)
    u = torch.randn(s.n, device="cuda", generator=g)
    v = torch.randn(s.n, device="cuda", generator=g)
    Bu = s.apply_precond(u).double()
    Bv = s.apply_precond(v).double()
    Buv = s.apply_precond(u + 2.0 * v).double()
    s.close()
    uv, vu = float(u.double() @ Bv), float(v.double() @ Bu)
    scale = float(u.double().abs() @ Bv.abs())
    print("<u, Bv> %.9g, <v, Bu> %.9g" % (uv, vu), flush=True)
    assert abs(uv - vu) <= 1e-5 * scale
    assert float(u.double() @ Bu) > 0 and float(v.double() @ Bv) > 0
    assert float((Buv - (Bu + 2.0 * Bv)).abs().max()) <= 1e-5 * float(Buv.abs().max())


@pytest.mark.parametrize("dims,mg", [((28, 27, 27), False), ((28, 28, 27), True)])
def test_auto_threshold(dims, mg):
    # AUTO takes the multigrid form from 2^17 even-band unknowns on: P3 on
    # 28 x 27 x 27 holds 127,036 of them, on 28 x 28 x 27 131,683
    print("case auto-threshold dims=%s" % (dims,), flush=True)
    m = config_small(3, dims, seed=71, sigma_range=(1.0, 40.0), albedo_range=(0.5, 0.99), sigma_t_min=1.0)
    s = solver(m)
    assert (s.even_unknowns() >= 1 << 17) == mg
    rhs = s.rhs_from_q00(dev(m.q00[0]))
    xa, ia = s.solve(rhs, tol=1e-8)
    xv, iv = s.solve(rhs, tol=1e-8, variant="schur_mg" if mg else "schur")
    s.close()
    assert ia["status"] == 0 and ia["inner_iters"] == iv["inner_iters"] and torch.equal(xa, xv)
