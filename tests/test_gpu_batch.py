"""GPU parity of the batched solve (pn_batch_*) and of the launch autotuner.

Every system of a batch (problem x right-hand side) must (i) meet the
requested FP64 relative residual, checked by the oracle's assembled matrix,
(ii) lie within a relative L2 error of 1e-5 of the oracle's solution, and
(iii) equal bitwise the single-system pn_solve of the same system with the
same launch shape (the batch runs the same arithmetic per system).
"""
import numpy as np
import pytest
import torch

from oracle.assemble import assemble, rhs_isotropic
from oracle.solve import cgls, direct
from synth import config_batch, config_small

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def problems(media):
    return [(m.order, m.dims, dev(m.sigma_t), dev(m.albedo), m.g, m.sigma_t_min, m.bc) for m in media]


def packed_rhs(lay, q00):
    b = torch.zeros(lay.n, dtype=torch.float32, device="cuda")
    b[lay.offset[0]:lay.offset[1]] = dev(q00).reshape(-1)
    return b


def oracle_solution(A, b):
    if A.shape[0] <= 20000:
        return direct(A, b)
    AT = A.T.tocsr()
    u, info = cgls(lambda v: A @ v, lambda v: AT @ v, b, tol=1e-13)
    assert info["rel_residual"] <= 1e-12
    return u


def single_solve(m, rhs, **kw):
    from paper_1807_00410_amd.solver import Solver
    s = Solver(m.order, m.dims, dev(m.sigma_t), dev(m.albedo), g=m.g, sigma_t_min=m.sigma_t_min, bc=m.bc)
    x, info = s.solve(rhs, **kw)
    z = s.zchunk()
    s.close()
    return x, info, z


def test_batch_mixed_orders_matches_single_and_oracle():
    from paper_1807_00410_amd.solver import Batch, tune_cache_clear
    tune_cache_clear()
    nrhs = 3
    media = config_batch(seed=5, nmedia=5, nrhs=nrhs, sizes=(6, 8, 11), orders=(1, 3, 5, 7))
    assert sorted({m.order for m in media}) == [1, 3, 5, 7]
    with Batch(problems(media), nrhs) as B:
        rhs = [packed_rhs(B.layouts[p], q) for p, m in enumerate(media) for q in m.q00]
        assert B.unknowns == sum(B.layouts[p].n for p in range(len(media))) * nrhs
        print("batch: %d systems, %d unknowns" % (len(rhs), B.unknowns), flush=True)
        xs, infos = B.solve(rhs, tol=1e-8)
        zs = [B.zchunk(p) for p in range(len(media))]
    for p, m in enumerate(media):
        A, lay = assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=m.bc)
        for r in range(nrhs):
            i = p * nrhs + r
            b = rhs_isotropic(lay, m.q00[r])
            u = oracle_solution(A, b)
            xv = xs[i].cpu().numpy()
            res = np.linalg.norm(b - A @ xv) / np.linalg.norm(b)
            err = np.linalg.norm(xv - u) / np.linalg.norm(u)
            print("system %d (P%d %s): iters=%d outer=%d res=%.3g err=%.3g" % (
                i, m.order, m.dims, infos[i]["inner_iters"], infos[i]["outer_iters"], res, err), flush=True)
            assert infos[i]["status"] == 0
            assert res <= 1.01e-8
            assert abs(res - infos[i]["rel_residual"]) <= 1e-11
            assert err <= 1e-5
            # the batch's default inner solver is the equilibrated CG
            x1, info1, z1 = single_solve(m, rhs[i], tol=1e-8, variant="cg_eq")
            assert z1 == zs[p]
            assert info1["inner_iters"] == infos[i]["inner_iters"]
            assert info1["outer_iters"] == infos[i]["outer_iters"]
            assert torch.equal(x1, xs[i])


def test_batch_zero_rhs_and_limits():
    from paper_1807_00410_amd.solver import Batch
    media = [config_small(3, (7, 6, 5), seed=1, nrhs=2), config_small(1, (9, 8, 7), seed=2, nrhs=2)]
    with Batch(problems(media), 2) as B:
        rhs = [packed_rhs(B.layouts[p], q) for p, m in enumerate(media) for q in m.q00]
        rhs[1].zero_()
        x0 = [torch.full((B.layouts[i // 2].n,), 5.0, dtype=torch.float64, device="cuda") for i in range(4)]
        xs, infos = B.solve(rhs, x=x0, tol=1e-8)
        assert [d["status"] for d in infos] == [0, 0, 0, 0]
        assert torch.count_nonzero(xs[1]) == 0
        # a tight iteration limit: every system reports "not converged", x stays finite
        xs, infos = B.solve(rhs, tol=1e-12, max_iter=5, raise_on_fail=False)
        assert infos[0]["status"] == 5 and infos[2]["status"] == 5 and infos[3]["status"] == 5
        assert infos[1]["status"] == 0
        assert all(torch.isfinite(v).all() for v in xs)
        # non-finite right-hand side
        from paper_1807_00410_amd.solver import PnError
        rhs[2][3] = float("nan")
        with pytest.raises(PnError) as e:
            B.solve(rhs, tol=1e-8)
        assert e.value.status == 4


def test_batch_use_guess_continues():
    from paper_1807_00410_amd.solver import Batch
    media = [config_small(5, (6, 5, 7), seed=3, nrhs=2)]
    with Batch(problems(media), 2) as B:
        rhs = [packed_rhs(B.layouts[0], q) for q in media[0].q00]
        xs, _ = B.solve(rhs, tol=1e-5)
        xs, infos = B.solve(rhs, x=xs, tol=1e-8, use_guess=True)
        for d in infos:
            assert d["status"] == 0 and d["history"][0] <= 1.01e-5


def test_autotune_and_cache():
    import os
    import tempfile
    from paper_1807_00410_amd.solver import (Batch, Solver, tune_cache_clear, tune_cache_load, tune_cache_save,
                                             tune_cache_size)
    tune_cache_clear()
    m = config_small(5, (20, 17, 23), seed=4)
    s = Solver(5, m.dims, dev(m.sigma_t), dev(m.albedo), g=m.g, sigma_t_min=m.sigma_t_min)
    x = dev(np.random.default_rng(1).normal(size=s.n))
    y0 = s.apply(x)
    z, ms = s.autotune(iters=3)
    assert z >= 1 and ms > 0 and s.zchunk() == z
    assert torch.equal(y0, s.apply(x))  # the launch shape never changes results
    assert tune_cache_size() == 1
    path = os.path.join(tempfile.mkdtemp(), "tune.txt")
    tune_cache_save(path)
    tune_cache_clear()
    tune_cache_load(path)
    assert tune_cache_size() == 1
    s2 = Solver(5, m.dims, dev(m.sigma_t), dev(m.albedo), g=m.g, sigma_t_min=m.sigma_t_min)
    assert s2.zchunk() == z  # setup takes the cached shape
    s2.close()
    s.close()
    # a tuned batch: shapes from the cache (tuning the shapes it lacks)
    media = [m, config_small(3, (9, 9, 9), seed=6)]
    with Batch(problems(media), 1, tune=True) as B:
        assert B.zchunk(0) == z
        assert tune_cache_size() == 2
        ms_b = B.bench_apply(iters=3)
        assert ms_b > 0
        rhs = [packed_rhs(B.layouts[p], mm.q00[0]) for p, mm in enumerate(media)]
        xs, infos = B.solve(rhs, tol=1e-8)
        assert all(d["status"] == 0 for d in infos)
    tune_cache_clear()


@pytest.mark.parametrize("variant", ["cgls", "cg", "cg_eq"])
def test_batch_variants_match_single(variant):
    # every Krylov variant of the batch equals pn_solve's bitwise
    from paper_1807_00410_amd.solver import Batch
    media = [config_small(5, (7, 6, 8), seed=8, nrhs=2), config_small(3, (9, 7, 6), seed=9, nrhs=2)]
    with Batch(problems(media), 2) as B:
        rhs = [packed_rhs(B.layouts[p], q) for p, m in enumerate(media) for q in m.q00]
        xs, infos = B.solve(rhs, tol=1e-8, variant=variant)
    for p, m in enumerate(media):
        A, lay = assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=m.bc)
        for r in range(2):
            i = p * 2 + r
            x1, info1, _ = single_solve(m, rhs[i], tol=1e-8, variant=variant)
            assert infos[i]["status"] == 0 and info1["inner_iters"] == infos[i]["inner_iters"]
            assert torch.equal(x1, xs[i])
            b = rhs_isotropic(lay, m.q00[r])
            assert np.linalg.norm(b - A @ xs[i].cpu().numpy()) / np.linalg.norm(b) <= 1.01e-8


def test_batch_problem_context_refuses_workspace_calls():
    """A batch problem's context has no Krylov workspace: every entry point
    that would need it returns PN_ERR_ARG on the host, launching nothing."""
    import ctypes as C
    from paper_1807_00410_amd import _lib as L
    from paper_1807_00410_amd.solver import Batch
    m = config_small(3, (5, 4, 3), seed=4)
    lib = L.load()
    with Batch(problems([m]), 1) as B:
        ctx = lib.pn_batch_problem(B.b, 0)
        assert ctx
        n = B.layouts[0].n
        x = torch.zeros(n, dtype=torch.float32, device="cuda")
        y = torch.zeros(n, dtype=torch.float32, device="cuda")
        x64 = torch.zeros(n, dtype=torch.float64, device="cuda")
        y64 = torch.zeros(n, dtype=torch.float64, device="cuda")
        p = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
        ms = C.c_double()
        rel = C.c_double()
        calls = [
            lib.pn_apply(ctx, p(x), p(y), 0),
            lib.pn_row_weights(ctx, p(y)),
            lib.pn_apply64(ctx, p(x64), p(y64), 1),
            lib.pn_residual64(ctx, p(x), p(x64), p(y64), C.byref(rel)),
            lib.pn_solve(ctx, p(x), p(x64), C.c_double(1e-8), None, None),
            lib.pn_bench_apply(ctx, 1, 0, C.byref(ms)),
            lib.pn_bench_kernel(ctx, 0, 1, C.byref(ms)),
            lib.pn_set_zchunk(ctx, 2),
            lib.pn_set_tiles(ctx, 32, 4, 0),
        ]
        assert calls == [L.PN_ERR_ARG] * len(calls)
        assert b"no Krylov workspace" in lib.pn_last_error(ctx)
        torch.cuda.synchronize()


def test_batch_multigrid_matches_single_and_oracle():
    # PN_VARIANT_SCHUR_MG: every system by the single-system multigrid
    # even-parity solve on its own right-hand side; equals pn_solve bitwise
    # (same launch shape) and reaches the oracle's answer
    from paper_1807_00410_amd.solver import Batch, Solver
    nrhs = 3
    media = config_batch(seed=9, nmedia=4, nrhs=nrhs, sizes=(8, 11, 16), orders=(1, 3, 5, 7))
    with Batch(problems(media), nrhs) as B:
        rhs = [packed_rhs(B.layouts[p], q) for p, m in enumerate(media) for q in m.q00]
        xs, infos = B.solve(rhs, tol=1e-8, variant="schur_mg")
        xs2, infos2 = B.solve(rhs, tol=1e-8, variant="schur_mg")  # graphs reused: same result
        zs = [B.zchunk(p) for p in range(len(media))]
    for p, m in enumerate(media):
        A, lay = assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=m.bc)
        s = Solver(m.order, m.dims, dev(m.sigma_t), dev(m.albedo), g=m.g, sigma_t_min=m.sigma_t_min, bc=m.bc)
        s.set_zchunk(zs[p])
        for r in range(nrhs):
            i = p * nrhs + r
            x1, i1 = s.solve(rhs[i], tol=1e-8, variant="schur_mg")
            assert infos[i]["status"] == 0 and i1["inner_iters"] == infos[i]["inner_iters"]
            assert torch.equal(x1, xs[i]) and torch.equal(xs[i], xs2[i])
            b = rhs_isotropic(lay, m.q00[r])
            u = oracle_solution(A, b)
            xv = xs[i].cpu().numpy()
            res = np.linalg.norm(b - A @ xv) / np.linalg.norm(b)
            err = np.linalg.norm(xv - u) / np.linalg.norm(u)
            print("system %d (P%d %s): iters=%d res=%.3g err=%.3g" % (i, m.order, m.dims, infos[i]["inner_iters"],
                                                                     res, err), flush=True)
            assert res <= 1.01e-8 and err <= 1e-5
        s.close()


def test_batch_multigrid_refused_with_a_neumann_problem():
    from paper_1807_00410_amd.solver import Batch, PnError
    media = [config_small(3, (6, 5, 4), seed=1, sigma_range=(2.0, 20.0), sigma_t_min=1.0),
             config_small(3, (6, 5, 4), seed=2, sigma_range=(2.0, 20.0), sigma_t_min=1.0, bc=2)]
    with Batch(problems(media), 1) as B:
        rhs = [packed_rhs(B.layouts[p], m.q00[0]) for p, m in enumerate(media)]
        with pytest.raises(PnError):
            B.solve(rhs, tol=1e-8, variant="schur_mg")
        xs, infos = B.solve(rhs, tol=1e-8)  # the batched CG path still serves the mixed batch
        assert all(d["status"] == 0 for d in infos)
