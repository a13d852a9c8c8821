"""GPU parity on the validation problems of section "Results", through the
C ABI, against the FP64 oracle:

* 2D checkerboard (7 x 7 unit blocks on 71 x 71 cells, one z-periodic cell):
  P1-P3 at full size within 1e-6 (rel-L2) of SuperLU; P4 and P5 at full size
  meet the residual 1e-10 of the oracle's own assembled matrix (SuperLU takes
  about a minute there) and P5 on 35 x 35 cells lies within 1e-6 of SuperLU.
  The coefficients with l + |m| odd vanish exactly (the problem is
  z-invariant).
* Point source (homogeneous sigma_t = 8, albedo 0.9, central 2^3 emission):
  P1-P5 on small grids within 1e-6 of SuperLU; at the full 80^3 the P1
  fluence equals the oracle's CDA solution within 1e-6 (the paper's "P1 is
  CDA"), and the P3 and P5 solutions are mirror-symmetric in every axis with
  the sign of each coefficient's staggering class, within 1e-6 of their
  largest magnitude, at the FP64 residual 1e-10.
The solves run to the residual 1e-10 the paper quotes for the checkerboard.
"""
import numpy as np
import pytest
import torch

from oracle.assemble import assemble, rhs_isotropic
from oracle.cda import cda_solve
from oracle.sh import coeff_lm
from oracle.solve import direct
from oracle.stagger import Layout
from synth import config_checkerboard, config_point_source

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def gpu_solve(m):
    from paper_1807_00410_amd.solver import Solver
    s = Solver(m.order, m.dims, dev(m.sigma_t), dev(m.albedo), g=m.g, sigma_t_min=m.sigma_t_min, bc=m.bc, h=m.h)
    x, info = s.solve(s.rhs_from_q00(dev(m.q00[0])), tol=TOL)
    xs = x.cpu().numpy()
    s.close()
    assert info["status"] == 0 and info["rel_residual"] <= TOL * 1.01, info
    return xs, Layout(m.order, m.dims, m.bc), info


def oracle_system(m):
    A, lay = assemble(m.order, m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, bc=m.bc, h=m.h or None)
    return A, lay, rhs_isotropic(lay, m.q00[0])


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def check_z_odd_zero(xs, lay):
    for k in range(lay.ncoeff):
        l, mm = coeff_lm(k)
        if (l + abs(mm)) % 2 == 1:
            assert np.abs(lay.view(xs, k)).max() == 0.0, "coefficient %d" % k


@pytest.mark.parametrize("order,n,check", [(1, 71, "direct"), (2, 71, "direct"), (3, 71, "direct"),
                                           (4, 71, "residual"), (5, 71, "residual"), (5, 35, "direct")])
def test_checkerboard(order, n, check):
    print("case checkerboard order=%d n=%d" % (order, n), flush=True)
    m = config_checkerboard(order, n=n)
    xs, lay, info = gpu_solve(m)
    A, olay, b = oracle_system(m)
    assert olay.n == lay.n
    if check == "direct":
        err = rel_l2(xs, direct(A, b))
        print("iters %d error %.3g" % (info["inner_iters"], err), flush=True)
        assert err <= 1e-6
    else:
        res = float(np.linalg.norm(b - A @ xs) / np.linalg.norm(b))
        print("iters %d oracle residual %.3g" % (info["inner_iters"], res), flush=True)
        assert res <= 1.01 * TOL
    check_z_odd_zero(xs, olay)
    if order == 1:  # the P1 fluence solves a diffusion problem (an M-matrix): positive; P_N with N > 1 need not be
        assert olay.view(xs, 0).min() > 0


@pytest.mark.parametrize("order,n", [(1, 16), (2, 12), (3, 12), (4, 8), (5, 8)])
def test_point_source_small_vs_direct(order, n):
    print("case point-source order=%d n=%d" % (order, n), flush=True)
    m = config_point_source(order, n=n)
    xs, lay, info = gpu_solve(m)
    A, _, b = oracle_system(m)
    err = rel_l2(xs, direct(A, b))
    print("iters %d error %.3g" % (info["inner_iters"], err), flush=True)
    assert err <= 1e-6


def test_point_source_80_p1_equals_cda():
    print("case point-source-80 P1 vs CDA", flush=True)
    m = config_point_source(1, n=80)
    xs, lay, info = gpu_solve(m)
    phi = cda_solve(m.dims, m.sigma_t, m.albedo, m.g, m.sigma_t_min, m.q00[0])
    err = rel_l2(lay.view(xs, 0), phi)
    print("iters %d error vs CDA %.3g" % (info["inner_iters"], err), flush=True)
    assert err <= 1e-6


@pytest.mark.parametrize("order", [3, 5])
def test_point_source_80_mirror_symmetry(order):
    print("case point-source-80 symmetry order=%d" % order, flush=True)
    m = config_point_source(order, n=80)
    xs, lay, info = gpu_solve(m)
    scale = np.abs(xs).max()
    worst = 0.0
    for k in range(lay.ncoeff):
        v = lay.view(xs, k)
        for d, ax in ((0, 2), (1, 1), (2, 0)):
            sign = -1.0 if lay.cls[k][d] == 1 else 1.0
            worst = max(worst, float(np.abs(v - sign * np.flip(v, axis=ax)).max()))
    print("iters %d symmetry defect %.3g of the largest magnitude" % (info["inner_iters"], worst / scale), flush=True)
    assert worst <= 1e-6 * scale
