"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances.  FP32 apply: every output element within
16 * eps32 * (|A| |x|)_i of the FP64 oracle (a bound on the rounding of the
differences, couplings, interpolation and the accumulation of <= 22 terms).
FP64 apply/residual: 64 * eps64 * (|A| |x|)_i.  Solves: the FP64 relative
residual computed by the oracle meets the requested tolerance, and the
relative L2 error against the oracle's direct solution is <= 1e-5.
"""
import numpy as np
import pytest
import torch

from oracle.apply import Operator, rows_of
from oracle.assemble import assemble, rhs_isotropic
from oracle.solve import cgls, direct
from synth import (config_p1_homogeneous, config_p3_fbm, config_p5_nebula, config_small,
                   config_uniform_periodic)

pytestmark = pytest.mark.gpu

EPS32 = float(np.finfo(np.float32).eps)
EPS64 = float(np.finfo(np.float64).eps)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def make_solver(m, **kw):
    from paper_1807_00410_amd.solver import Solver
    return Solver(m.order, m.dims, dev(m.sigma_t), dev(m.albedo), g=m.g, sigma_t_min=m.sigma_t_min, bc=m.bc, **kw)


def oracle_matrix(m):
    return assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=m.bc)


def magnitude_matrix(m):
    """|T| + diag(sigma_t + |g|^l sigma_s): the sizes of the terms of every row
    before the sigma_t - g^l sigma_s cancellation (the scale of a rounding
    bound for either side).  Assembled by the oracle with the albedo negated
    and |g|, which turns the diagonal difference into the sum."""
    M, _ = assemble(m.order, m.dims, m.sigma_t, -m.albedo, abs(m.g), m.sigma_t_min, bc=m.bc)
    return abs(M)


def check_layout(s, lay):
    assert s.n == lay.n
    assert s.layout.offset == [int(v) for v in lay.offset]
    assert s.layout.cls == [tuple(c) for c in lay.cls]
    assert s.layout.ext == [tuple(e) for e in lay.ext]


CASES = [
    (1, (37, 29, 23), 0), (1, (19, 17, 13), 1),
    (2, (21, 18, 15), 0),
    (3, (33, 27, 21), 0), (3, (16, 12, 10), 1),
    (4, (15, 14, 13), 0),
    (5, (21, 19, 17), 0), (5, (12, 10, 9), 1),
    (6, (11, 10, 9), 0),
    (7, (13, 12, 11), 0), (7, (8, 7, 6), 1),
    (3, (1, 1, 1), 0), (5, (2, 3, 1), 0), (1, (1, 1, 1), 1), (5, (3, 2, 4), 1),
]


@pytest.mark.parametrize("order,dims,bc", CASES)
@pytest.mark.parametrize("transpose", [False, True])
def test_apply_fp32_vs_oracle(order, dims, bc, transpose):
    print("case apply32 order=%d dims=%s bc=%d T=%d" % (order, dims, bc, transpose), flush=True)
    m = config_small(order, dims, seed=order * 7 + bc, bc=bc)
    A, lay = oracle_matrix(m)
    s = make_solver(m)
    check_layout(s, lay)
    x = np.random.default_rng(order).normal(size=lay.n).astype(np.float32)
    y = s.apply(dev(x), transpose=transpose).cpu().numpy().astype(np.float64)
    M = A.T.tocsr() if transpose else A
    Mag = magnitude_matrix(m)
    Mag = Mag.T.tocsr() if transpose else Mag
    ref = M @ x.astype(np.float64)
    bound = 16 * EPS32 * (Mag @ np.abs(x.astype(np.float64))) + 1e-30
    err = np.abs(y - ref)
    assert np.all(err <= bound), "max err/bound %g" % float((err / bound).max())
    s.close()


@pytest.mark.parametrize("order,dims,bc", [c for c in CASES if c[0] in (1, 3, 5, 7)])
def test_apply_fp64_vs_oracle(order, dims, bc):
    print("case apply64 order=%d dims=%s bc=%d" % (order, dims, bc), flush=True)
    m = config_small(order, dims, seed=order * 5 + bc, bc=bc)
    A, lay = oracle_matrix(m)
    s = make_solver(m)
    x = np.random.default_rng(order + 1).normal(size=lay.n)
    Mag = magnitude_matrix(m)
    for transpose in (False, True):
        y = s.apply64(dev(x, torch.float64), transpose=transpose).cpu().numpy()
        M = A.T.tocsr() if transpose else A
        ref = M @ x
        bound = 64 * EPS64 * ((Mag.T.tocsr() if transpose else Mag) @ np.abs(x)) + 1e-300
        assert np.all(np.abs(y - ref) <= bound)
    s.close()


def test_apply_deterministic_and_nan_poison_untouched():
    # run twice -> bitwise identical; output entries are all written (NaN poison gone)
    m = config_small(5, (17, 13, 11), seed=3)
    s = make_solver(m)
    x = dev(np.random.default_rng(0).normal(size=s.n))
    y1 = torch.full_like(x, float("nan"))
    y2 = torch.full_like(x, float("nan"))
    s.apply(x, y1)
    s.apply(x, y2)
    assert torch.isfinite(y1).all()
    assert torch.equal(y1, y2)
    # a buffer beyond the vector stays untouched
    big = torch.full((s.n + 1000,), 7.0, device="cuda")
    s.apply(x, big[:s.n])
    assert torch.all(big[s.n:] == 7.0)
    s.close()


def test_residual64_vs_oracle():
    m = config_small(3, (14, 11, 9), seed=4)
    A, lay = oracle_matrix(m)
    s = make_solver(m)
    rng = np.random.default_rng(2)
    x = rng.normal(size=lay.n)
    b = rhs_isotropic(lay, m.q00[0]).astype(np.float32)
    r = torch.empty(lay.n, dtype=torch.float64, device="cuda")
    rel = s.residual64(dev(b), dev(x, torch.float64), r)
    ref = b.astype(np.float64) - A @ x
    bound = 64 * EPS64 * (np.abs(b) + magnitude_matrix(m) @ np.abs(x))
    assert np.all(np.abs(r.cpu().numpy() - ref) <= bound)
    assert abs(rel - np.linalg.norm(ref) / np.linalg.norm(b.astype(np.float64))) < 1e-12 * rel
    s.close()


def oracle_solution(A, b):
    """Reference solution: SuperLU for small systems, the oracle's FP64 CGLS
    to a relative residual of 1e-13 otherwise (3D fill-in makes LU slow)."""
    if A.shape[0] <= 20000:
        return direct(A, b)
    AT = A.T.tocsr()
    u, info = cgls(lambda v: A @ v, lambda v: AT @ v, b, tol=1e-13)
    assert info["rel_residual"] <= 1e-12
    return u


def _solve_and_check(m, tol, precision, err_tol=1e-5, **kw):
    A, lay = oracle_matrix(m)
    b = rhs_isotropic(lay, m.q00[0])
    u = oracle_solution(A, b)
    s = make_solver(m)
    rhs = s.rhs_from_q00(dev(m.q00[0]))
    assert np.array_equal(rhs.cpu().numpy(), b.astype(np.float32))
    x, info = s.solve(rhs, tol=tol, precision=precision, **kw)
    xs = x.cpu().numpy()
    res = np.linalg.norm(b - A @ xs) / np.linalg.norm(b)
    err = np.linalg.norm(xs - u) / np.linalg.norm(u)
    print("solve %s %s: iters=%d outer=%d res=%.3g (gpu %.3g) err=%.3g t=%.3fs" % (
        m.name, precision, info["inner_iters"], info["outer_iters"], res, info["rel_residual"], err,
        info["seconds"]), flush=True)
    assert info["status"] == 0
    assert res <= tol * 1.01
    assert abs(res - info["rel_residual"]) <= 1e-3 * tol
    assert err <= err_tol
    s.close()
    return info


def test_solve_p1_homogeneous_fp64():
    # P1, 16^3, sigma_t = 10, albedo 0.9, central 2^3 emission, FP64 Krylov to 1e-10
    _solve_and_check(config_p1_homogeneous(16), 1e-10, "fp64", err_tol=1e-8)


def test_solve_p1_homogeneous_fp32_ir():
    _solve_and_check(config_p1_homogeneous(16), 1e-10, "fp32_ir", err_tol=1e-8)


@pytest.mark.parametrize("order,n", [(3, 16), (3, 20), (5, 12)])
def test_solve_small_fbm_fp32_ir(order, n):
    m = config_p3_fbm(n=n, seed=11, order=order)
    _solve_and_check(m, 1e-8, "fp32_ir")


def test_solve_small_nebula_fp32_ir():
    for g in (0.0, 0.5):
        m = config_p5_nebula(n=12, seed=5, g=g, order=5)
        _solve_and_check(m, 1e-8, "fp32_ir")


def test_uniform_periodic_closed_form():
    m = config_uniform_periodic(n=10, order=5, sigma_t=5.0, albedo=0.8, g=0.4, q=2.0)
    s = make_solver(m)
    rhs = s.rhs_from_q00(dev(m.q00[0]))
    x, info = s.solve(rhs, tol=1e-10, precision="fp64")
    xs = x.cpu().numpy()
    sa = float(np.float32(5.0)) * (1.0 - float(np.float32(0.8)))
    lay = s.layout
    np.testing.assert_allclose(xs[:lay.offset[1]], 2.0 / sa, rtol=1e-9)
    assert np.abs(xs[lay.offset[1]:]).max() < 1e-9
    s.close()


def test_zero_rhs_gives_zero():
    m = config_small(3, (6, 5, 4), seed=1)
    s = make_solver(m)
    x = torch.full((s.n,), 3.0, dtype=torch.float64, device="cuda")
    x, info = s.solve(torch.zeros(s.n, device="cuda"), x=x, tol=1e-8)
    assert info["status"] == 0 and torch.count_nonzero(x) == 0
    s.close()


def test_nonfinite_medium_and_rhs():
    from paper_1807_00410_amd.solver import PnError
    m = config_small(3, (6, 5, 4), seed=1)
    st = m.sigma_t.copy()
    st[2, 1, 3] = np.nan
    from paper_1807_00410_amd.solver import Solver
    with pytest.raises(PnError) as e:
        Solver(3, m.dims, dev(st), dev(m.albedo), g=m.g, sigma_t_min=m.sigma_t_min)
    assert e.value.status == 4
    s = make_solver(m)
    rhs = torch.zeros(s.n, device="cuda")
    rhs[5] = float("inf")
    with pytest.raises(PnError) as e:
        s.solve(rhs, tol=1e-8)
    assert e.value.status == 4
    s.close()


def test_vacuum_without_threshold_reports_not_converged():
    # sigma_t = 0 regions and no threshold: A is singular (the paper's vacuum case).
    m = config_small(3, (8, 8, 8), seed=2)
    st = m.sigma_t.copy()
    st[:, :, :4] = 0.0
    from paper_1807_00410_amd.solver import Solver
    s = Solver(3, m.dims, dev(st), dev(m.albedo), g=m.g, sigma_t_min=0.0)
    rhs = s.rhs_from_q00(dev(m.q00[0]))
    x, info = s.solve(rhs, tol=1e-12, max_iter=300, raise_on_fail=False)
    assert info["status"] == 5
    assert torch.isfinite(x).all()
    s.close()


def test_use_guess_continues_from_x():
    m = config_p3_fbm(n=12, seed=2, order=3)
    s = make_solver(m)
    rhs = s.rhs_from_q00(dev(m.q00[0]))
    x, info1 = s.solve(rhs, tol=1e-6)
    x, info2 = s.solve(rhs, x=x, tol=1e-8, use_guess=True)
    assert info2["status"] == 0 and info2["history"][0] <= 1.01e-6
    s.close()


@pytest.mark.parametrize("zchunk", [1, 3, 7, 1000])
def test_zchunk_variants_identical(zchunk):
    m = config_small(5, (14, 9, 11), seed=9)
    s = make_solver(m)
    x = dev(np.random.default_rng(3).normal(size=s.n))
    y0 = s.apply(x)
    s.set_zchunk(zchunk)
    y1 = s.apply(x)
    assert torch.equal(y0, y1)
    s.close()


def test_full_size_p5_apply_sampled_rows():
    # P5 on 128^3 (the nebula workload): sampled output rows against the oracle's
    # one-row-at-a-time evaluation.
    m = config_p5_nebula(n=128, seed=3, g=0.5)
    s = make_solver(m)
    rng = np.random.default_rng(0)
    x = rng.normal(size=s.n).astype(np.float32)
    y = s.apply(dev(x)).cpu().numpy()
    rows = np.concatenate([rng.integers(0, s.n, 3000), [0, s.n - 1]])
    args = (5, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min)
    ref = rows_of(*args, x.astype(np.float64), rows)
    bound = 16 * EPS32 * rows_of(*args, x.astype(np.float64), rows, absolute=True)
    assert np.all(np.abs(y[rows] - ref) <= bound)
    s.close()


@pytest.mark.parametrize("order,n", [(3, 16), (5, 12), (1, 20)])
def test_solve_cg_normal_equations_variant(order, n):
    # CG on the normal equations with the recursive normal residual
    # (s -= alpha A^T q in the register-window stencil): same answer to 1e-5
    m = config_p3_fbm(n=n, seed=13, order=order)
    _solve_and_check(m, 1e-8, "fp32_ir", variant="cg")


@pytest.mark.parametrize("order,dims,bc", [(3, (9, 7, 8), 0), (5, (7, 6, 8), 0), (7, (6, 5, 7), 0),
                                           (2, (6, 7, 5), 1), (5, (5, 6, 4), 1)])
def test_row_weights_are_inverse_squared_row_norms(order, dims, bc):
    # W of the equilibrated variant against the rows of the oracle's assembled
    # matrix: 1 / ||row||^2 wherever the row has all its entries, and no larger
    # where a vacuum boundary removed some (FP32 reciprocal: 1e-6 relative)
    m = config_small(order, dims, seed=order + 60, bc=bc)
    A, lay = oracle_matrix(m)
    s = make_solver(m)
    w = s.row_weights().cpu().numpy().astype(np.float64)
    s.close()
    A = A.tocsr()
    rn2 = np.asarray(A.multiply(A).sum(axis=1)).ravel()
    nnz = np.diff(A.indptr)
    full = np.zeros(lay.n, dtype=bool)
    for k in range(len(lay.offset) - 1):
        sl = slice(lay.offset[k], lay.offset[k + 1])
        full[sl] = nnz[sl] == nnz[sl].max()
    assert full.sum() > 0
    ref = 1.0 / rn2
    assert np.all(np.abs(w[full] - ref[full]) <= 1e-6 * ref[full])
    assert np.all(w <= ref * (1 + 1e-6))
    if bc == 1:
        assert full.all()


@pytest.mark.parametrize("order,n,bc", [(3, 16, 0), (5, 12, 0), (1, 20, 0), (3, 10, 1)])
def test_solve_equilibrated_cg_variant(order, n, bc):
    # CG on the row-equilibrated normal equations: the oracle's answer, with
    # the true (unweighted) FP64 residual at the tolerance
    if bc == 1:
        m = config_uniform_periodic(n=n, order=order, sigma_t=5.0, albedo=0.8, g=0.4, q=2.0)
    else:
        m = config_p3_fbm(n=n, seed=13, order=order)
    i_eq = _solve_and_check(m, 1e-8, "fp32_ir", variant="cg_eq")
    i_plain = _solve_and_check(m, 1e-8, "fp32_ir", variant="cg")
    print("iterations: equilibrated %d, plain %d" % (i_eq["inner_iters"], i_plain["inner_iters"]))
    # AUTO is the even-parity Schur form on the register-window stencil, with
    # the multigrid preconditioner for odd orders of at least 2^17 even-band
    # unknowns
    s = make_solver(m)
    rhs = s.rhs_from_q00(dev(m.q00[0]))
    xa, ia = s.solve(rhs, tol=1e-8)
    big = s.layout.order % 2 == 1 and s.even_unknowns() >= 1 << 17
    xe, ie = s.solve(rhs, tol=1e-8, variant="schur_mg" if big else "schur")
    assert ia["inner_iters"] == ie["inner_iters"] and torch.equal(xa, xe)
    s.close()


def test_bench_kernel_timings_and_state_reset():
    # every Krylov-loop kernel can be timed in its in-loop form; a solve after
    # the timings (which overwrite the workspace and the device scalars)
    # still reaches the oracle's answer
    from paper_1807_00410_amd.solver import PnError
    m = config_p3_fbm(n=16, seed=13, order=3)
    A, lay = oracle_matrix(m)
    b = rhs_isotropic(lay, m.q00[0])
    s = make_solver(m)
    rhs = s.rhs_from_q00(dev(m.q00[0]))
    s.solve(rhs, tol=1e-8)
    for k in ("apply", "apply_t", "apply_eq", "supd", "update"):
        assert s.bench_kernel(k, 3) > 0.0
    x, info = s.solve(rhs, tol=1e-8)
    xs = x.cpu().numpy()
    assert info["status"] == 0 and np.linalg.norm(b - A @ xs) / np.linalg.norm(b) <= 1.01e-8
    with pytest.raises(PnError):
        s._check(s.lib.pn_bench_kernel(s.ctx, 7, 3, None))
    s.set_tiles(32, 4)
    assert s.bench_kernel("apply", 2) > 0.0
    with pytest.raises(PnError):
        s.bench_kernel("supd", 2)
    s.close()


def test_equilibrated_variant_rejects_tiled_stencil_and_fp64():
    from paper_1807_00410_amd.solver import PnError
    m = config_small(3, (12, 10, 9), seed=3)
    s = make_solver(m)
    rhs = s.rhs_from_q00(dev(m.q00[0]))
    with pytest.raises(PnError) as e:
        s.solve(rhs, tol=1e-6, precision="fp64", variant="cg_eq")
    assert e.value.status == 1
    s.set_tiles(32, 4)
    with pytest.raises(PnError):
        s.solve(rhs, tol=1e-6, variant="cg_eq")
    x, info = s.solve(rhs, tol=1e-8)  # AUTO falls back to plain CG on the tiled stencil
    assert info["status"] == 0
    s.close()


@pytest.mark.parametrize("order,dims,tiles", [(3, (21, 18, 15), (32, 4)), (5, (17, 19, 13), (32, 4)),
                                              (1, (33, 9, 7), (64, 4)), (7, (9, 8, 7), (16, 3))])
def test_lds_tiled_stencil_apply_and_solve(order, dims, tiles):
    # the opt-in LDS-tiled stencil: apply within the FP32 bound of the oracle,
    # and the CG solve on it reaches the oracle's answer
    print("case lds order=%d dims=%s tiles=%s" % (order, dims, tiles), flush=True)
    from paper_1807_00410_amd.solver import PnError
    m = config_small(order, dims, seed=order + 40)
    A, lay = oracle_matrix(m)
    s = make_solver(m)
    s.set_tiles(*tiles)
    assert s.tiles()[:2] == tiles
    x = np.random.default_rng(order).normal(size=lay.n).astype(np.float32)
    Mag = magnitude_matrix(m)
    for transpose in (False, True):
        y = s.apply(dev(x), transpose=transpose).cpu().numpy().astype(np.float64)
        M = A.T.tocsr() if transpose else A
        ref = M @ x.astype(np.float64)
        bound = 16 * EPS32 * ((Mag.T.tocsr() if transpose else Mag) @ np.abs(x.astype(np.float64))) + 1e-30
        assert np.all(np.abs(y - ref) <= bound)
    b = rhs_isotropic(lay, m.q00[0])
    u = oracle_solution(A, b)
    xs, info = s.solve(s.rhs_from_q00(dev(m.q00[0])), tol=1e-8, variant="cg")
    xs = xs.cpu().numpy()
    assert info["status"] == 0
    assert np.linalg.norm(b - A @ xs) / np.linalg.norm(b) <= 1.01e-8
    assert np.linalg.norm(xs - u) / np.linalg.norm(u) <= 1e-5
    with pytest.raises(PnError):
        s.set_tiles(300, 300)
    s.set_tiles(0, 0)
    assert s.tiles()[:2] == (0, 0)
    s.close()
