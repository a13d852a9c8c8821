"""Accuracy at full size: the GPU solve of the P3 64^3 fBm workload (FP32
Krylov + FP64 refinement to an FP64 relative residual of 1e-8) against the
oracle's own FP64 CGLS solution of the same system, solved to 1e-12 by
tests/golden/make_references.py (C/OpenMP oracle, stored in FP32) -- the
relative L2 error must be at most 1e-5.  The stored reference's metadata is
checked too (its residual, its workload)."""
import json
import os

import numpy as np
import pytest
import torch

from synth import config_p3_fbm

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_p3_64_solution_within_1e5_of_oracle():
    from paper_1807_00410_amd.solver import Solver
    with open(os.path.join(GOLDEN, "ref_p3_64.json")) as fh:
        meta = json.load(fh)
    ref = np.load(os.path.join(GOLDEN, "ref_p3_64.npz"))["u"].astype(np.float64)
    assert meta["rel_residual"] <= 1e-11 and meta["dims"] == [64, 64, 64] and meta["order"] == 3
    m = config_p3_fbm(n=64, seed=1)
    print("full-size parity: %s, %d unknowns" % (m.name, ref.size), flush=True)
    s = Solver(m.order, m.dims, torch.as_tensor(m.sigma_t).cuda(), torch.as_tensor(m.albedo).cuda(), g=m.g,
               sigma_t_min=m.sigma_t_min)
    assert s.n == ref.size
    x, info = s.solve(s.rhs_from_q00(torch.as_tensor(m.q00[0]).cuda()), tol=1e-8)
    s.close()
    xs = x.cpu().numpy()
    err = np.linalg.norm(xs - ref) / np.linalg.norm(ref)
    print("rel residual %.3g, %d iterations, rel-L2 error vs oracle %.3g" % (
        info["rel_residual"], info["inner_iters"], err), flush=True)
    assert info["rel_residual"] <= 1e-8
    assert err <= 1e-5
