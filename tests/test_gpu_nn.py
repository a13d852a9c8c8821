"""GPU parity of the network kernels (BF16 matrix-core convolutions, pooling,
upsampling, Adam) and of the whole U-Net's forward pass and gradients against
the FP64 network oracle (oracle/nn.py).

Inputs are drawn from values that bfloat16 holds exactly (k / 64 with
|k| <= 128), so both sides see the same numbers.  Tolerances: FP32
accumulation of at most 27*32 exact products per output (and of V products
per weight gradient) -- 1e-5 of the sum of absolute terms; bfloat16-rounded
outputs one more rounding (2^-8 relative).  The whole network stores every
activation and gradient in bfloat16; the oracle rounds its activations at the
same points (quant=True) and keeps FP64 gradients, so the network gradients
are compared in relative L2 norm (3e-2 per convolution).
"""
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


def exact(rng, shape, scale=1.0):
    return rng.integers(-128, 129, size=shape).astype(np.float64) / 64.0 * scale


def bf(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).to(torch.bfloat16).cuda()


def f32(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).cuda()


def host(t):
    return t.float().cpu().numpy().astype(np.float64)


SHAPES = [(1, 8, 8, 8), (2, 6, 5, 7), (1, 13, 3, 9), (3, 4, 4, 2)]


@pytest.mark.parametrize("B,nx,ny,nz", SHAPES)
def test_conv3d_forward(B, nx, ny, nz):
    from paper_1807_00410_amd import net as N
    rng = np.random.default_rng(nx * 7 + ny)
    x = exact(rng, (B, nz, ny, nx, KC))
    w = exact(rng, (27, KC, KC), 1.0 / 16)
    b = exact(rng, KC)
    ref = O.conv3d(x, w, b)
    mag = O.conv3d(np.abs(x), np.abs(w), np.abs(b))
    y = host(N.conv3d(bf(x), bf(w), f32(b), relu=False, out_f32=True))
    assert np.all(np.abs(y - ref) <= 1e-5 * mag + 1e-30)
    yr = host(N.conv3d(bf(x), bf(w), f32(b), relu=True, out_f32=False))
    r = np.maximum(ref, 0.0)
    assert np.all(np.abs(yr - r) <= 2.0 ** -8 * np.abs(r) + 1e-5 * mag + 1e-30)


@pytest.mark.parametrize("B,nx,ny,nz", SHAPES)
def test_conv3d_dgrad_and_wgrad(B, nx, ny, nz):
    from paper_1807_00410_amd import net as N
    rng = np.random.default_rng(nx + 11 * nz)
    x = exact(rng, (B, nz, ny, nx, KC))
    g = exact(rng, (B, nz, ny, nx, KC), 1.0 / 8)
    w = exact(rng, (27, KC, KC), 1.0 / 16)
    ref = O.conv3d_dgrad(g, w)
    mag = O.conv3d_dgrad(np.abs(g), np.abs(w))
    dx = host(N.conv3d_dgrad(bf(g), bf(w)))
    assert np.all(np.abs(dx - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * mag + 1e-30)
    dw_ref, db_ref = O.conv3d_wgrad(x, g)
    dw_mag, db_mag = O.conv3d_wgrad(np.abs(x), np.abs(g))
    dw, db = N.conv3d_wgrad(bf(x), bf(g))
    assert np.all(np.abs(host(dw) - dw_ref) <= 1e-5 * dw_mag + 1e-30)
    assert np.all(np.abs(host(db) - db_ref) <= 1e-5 * db_mag + 1e-30)


def test_pool_upsample_and_adjoints():
    from paper_1807_00410_amd import net as N
    rng = np.random.default_rng(3)
    x = exact(rng, (2, 6, 4, 8, KC))
    s = exact(rng, (2, 6, 4, 8, KC))
    c = exact(rng, (2, 3, 2, 4, KC))
    p = host(N.pool2(bf(x)))
    ref = O.pool2(x)
    assert np.all(np.abs(p - ref) <= 2.0 ** -8 * np.abs(ref))
    u = host(N.up2_add(bf(c), bf(s)))
    ref = O.up2(c) + s
    assert np.all(np.abs(u - ref) <= 2.0 ** -8 * np.abs(ref))
    np.testing.assert_array_equal(host(N.up2_add(bf(c))), O.up2(c))
    ub = host(N.up2_bwd(bf(x)))
    ref = O.up2_bwd(x)
    assert np.all(np.abs(ub - ref) <= 2.0 ** -8 * np.abs(ref))
    pb = host(N.pool2_bwd_add(bf(c), bf(s)))
    ref = O.pool2_bwd(c) + s
    assert np.all(np.abs(pb - ref) <= 2.0 ** -8 * np.abs(ref))


def test_adam_matches_oracle():
    from paper_1807_00410_amd import net as N
    rng = np.random.default_rng(4)
    n = 5000
    w = rng.normal(size=n)
    m = rng.normal(size=n) * 0.1
    v = np.abs(rng.normal(size=n)) * 0.01
    g = rng.normal(size=n)
    w32, m32, v32, g32 = (np.float32(a).astype(np.float64) for a in (w, m, v, g))
    wr, mr, vr = O.adam(w32, g32, m32, v32, 3, 1e-3)
    tw, tm, tv = f32(w32), f32(m32), f32(v32)
    N.adam(tw, f32(g32), tm, tv, 3, 1e-3)
    # FP32 rounding relative to the sizes of the terms (m and v may cancel)
    assert np.all(np.abs(host(tm) - mr) <= 1e-6 * (0.9 * np.abs(m32) + 0.1 * np.abs(g32)))
    assert np.all(np.abs(host(tv) - vr) <= 1e-6 * (0.999 * v32 + 0.001 * g32 * g32))
    step = np.abs(wr - w32)
    assert np.all(np.abs(host(tw) - wr) <= 1e-6 * np.abs(w32) + 1e-5 * step)


def _params(seed):
    rng = np.random.default_rng(seed)
    flat = np.zeros(O.NCONV * (27 * KC * KC + KC), dtype=np.float32)
    ps = []
    for i in range(O.NCONV):
        w = (rng.normal(size=(27, KC, KC)) * np.sqrt(2.0 / (27 * KC))).astype(np.float32)
        b = (rng.normal(size=KC) * 0.05).astype(np.float32)
        o = i * (27 * KC * KC + KC)
        flat[o:o + 27 * KC * KC] = w.reshape(-1)
        flat[o + 27 * KC * KC:o + 27 * KC * KC + KC] = b
        ps.append((O.bf16_round(w), b.astype(np.float64)))
    return flat, ps


@pytest.mark.parametrize("B,n", [(1, 8), (2, 16)])
def test_unet_forward_and_gradients(B, n):
    from paper_1807_00410_amd.net import Net
    flat, ps = _params(5)
    rng = np.random.default_rng(6)
    x = exact(rng, (B, n, n, n, KC), 0.5)
    t = exact(rng, (B, n, n, n, 16), 0.25)
    net = Net(seed=1)
    net.set_params(flat)
    y = host(net.forward(bf(x)))
    yr, cache = O.unet_forward(ps, x, quant=True)
    rel = np.linalg.norm(y - yr) / np.linalg.norm(yr)
    print("forward rel L2 %.3g" % rel, flush=True)
    assert rel <= 1e-2
    loss = net.train_step(bf(x), bf(t), 0.0)
    yp = np.zeros_like(yr)
    yp[..., :16] = t
    lr_, dy = O.mse(yr, yp, 16)
    assert abs(loss - lr_) <= 2e-2 * lr_
    g = net.grads()
    grads = O.unet_backward(ps, cache, dy)
    per = 27 * KC * KC + KC
    for i in range(O.NCONV):
        gw = g[i * per:i * per + 27 * KC * KC].astype(np.float64)
        gb = g[i * per + 27 * KC * KC:(i + 1) * per].astype(np.float64)
        rw = grads[i][0].reshape(-1)
        rb = grads[i][1]
        ew = np.linalg.norm(gw - rw) / np.linalg.norm(rw)
        eb = np.linalg.norm(gb - rb) / max(np.linalg.norm(rb), 1e-30)
        print("conv %2d: dW rel %.3g  db rel %.3g" % (i, ew, eb), flush=True)
        assert ew <= 3e-2 and eb <= 3e-2
    net.close()


def test_training_reduces_loss_and_save_load(tmp_path):
    from paper_1807_00410_amd.net import Net
    rng = np.random.default_rng(7)
    xh = exact(rng, (2, 16, 16, 16, KC), 0.5)
    x = bf(xh)
    t = bf(0.3 + 0.5 * xh[..., :16])  # a target the network can represent
    net = Net(seed=2)
    l0 = net.train_step(x, t, 5e-3)
    for _ in range(40):
        l1 = net.train_step(x, t, 5e-3)
    print("loss %.4g -> %.4g" % (l0, l1))
    assert l1 < 0.7 * l0
    y1 = net.forward(x)
    path = tmp_path / "w.bin"
    net.save(path)
    net2 = Net(seed=99)
    net2.load(path)
    assert torch.equal(net2.forward(x), y1)
    assert np.array_equal(net2.params(), net.params())
    net.close()
    net2.close()


def test_net_load_rejects_foreign_files(tmp_path):
    from paper_1807_00410_amd.net import Net, NetError
    net = Net(seed=4)
    p0 = net.params()
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"not a network file")
    with pytest.raises(NetError) as e:
        net.load(bad)
    assert e.value.status == 1
    with pytest.raises(NetError):
        net.load(tmp_path / "missing.bin")
    assert np.array_equal(net.params(), p0)  # a failed load leaves the parameters
    net.close()


def test_net_train_loop():
    from paper_1807_00410_amd.net import Net
    rng = np.random.default_rng(9)
    xs, ts = [], []
    for _ in range(8):
        xh = exact(rng, (1, 8, 8, 8, KC), 0.5)
        xs.append(bf(xh))
        ts.append(bf(0.3 + 0.5 * xh[..., :16]))
    net = Net(seed=5)
    first = np.mean([net.train_step(xs[i], ts[i], 0.0) for i in range(8)])
    last = net.train(xs, ts, epochs=15, batch=2, lr=5e-3, seed=1)
    print("train loop: loss %.4g -> %.4g" % (first, last))
    assert last < 0.7 * first
    net.close()
