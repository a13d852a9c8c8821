"""The allocation-free weight gradient (pn_nn_conv3d_wgrad_noalloc) against
the allocating entry point (pn_nn_conv3d_wgrad) through the C ABI: two calls
in a row, the second on a smaller volume (its partial-sum blocks are a prefix
of the first call's, so stale scratch contents would show), each bitwise equal
to the allocating call (same kernels, same block split, same summation
order) and within the FP32 accumulation bound of the FP64 network oracle.
A volume beyond the scratch capacity is refused on the host."""
import numpy as np
import pytest
import torch

from oracle import nn as O

pytestmark = pytest.mark.gpu
KC = 32


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _exact(rng, shape):
    return rng.integers(-128, 129, size=shape).astype(np.float64) / 64.0


def _bf(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).to(torch.bfloat16).cuda()


def test_wgrad_noalloc_matches_allocating_entry_point():
    from paper_1807_00410_amd import net as N
    rng = np.random.default_rng(11)
    # (2, 16x16x16): 8192 voxels, 32 partial blocks; then (1, 10x6x8): 480 voxels, 2 blocks
    for B, nx, ny, nz in ((2, 16, 16, 16), (1, 10, 6, 8)):
        print("wgrad_noalloc B=%d nx=%d ny=%d nz=%d" % (B, nx, ny, nz), flush=True)
        x = _exact(rng, (B, nz, ny, nx, KC))
        g = _exact(rng, (B, nz, ny, nx, KC))
        xb, gb = _bf(x), _bf(g)
        dw = torch.full((27, KC, KC), float("nan"), dtype=torch.float32, device="cuda")
        db = torch.full((KC,), float("nan"), dtype=torch.float32, device="cuda")
        N.conv3d_wgrad_noalloc(xb, gb, dw, db)
        torch.cuda.synchronize()
        dw_ref, db_ref = N.conv3d_wgrad(xb, gb)
        torch.cuda.synchronize()
        assert torch.equal(dw, dw_ref) and torch.equal(db, db_ref)
        # and the function itself: FP32 sums of exact products vs the FP64 oracle
        ow, ob = O.conv3d_wgrad(x, g)
        mw, mb = O.conv3d_wgrad(np.abs(x), np.abs(g))
        assert np.all(np.abs(dw.cpu().numpy() - ow) <= 1e-5 * mw + 1e-30)
        assert np.all(np.abs(db.cpu().numpy() - ob) <= 1e-5 * mb + 1e-30)


def test_wgrad_noalloc_rejects_volume_beyond_scratch():
    from paper_1807_00410_amd import net as N
    x = torch.zeros((1, 33, 32, 32, KC), dtype=torch.bfloat16, device="cuda")  # 33792 voxels > 32768
    dw = torch.zeros((27, KC, KC), dtype=torch.float32, device="cuda")
    db = torch.zeros(KC, dtype=torch.float32, device="cuda")
    with pytest.raises(N.NetError) as e:
        N.conv3d_wgrad_noalloc(x, x, dw, db)
    assert "at most 128" in str(e.value)
