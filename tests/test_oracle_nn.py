"""Pins of the network oracle (oracle/nn.py): brute-force loops, closed forms,
adjoint identities and central finite differences, all on the CPU."""
import numpy as np

from oracle import nn


def rnd(*shape, seed=0):
    return np.random.default_rng(seed).normal(size=shape)


def test_bf16_round_ties_to_even():
    one = 1.0
    assert nn.bf16_round(one) == 1.0
    assert nn.bf16_round(1.0 + 2.0 ** -8) == 1.0                      # halfway, even stays
    assert nn.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6      # halfway, odd rounds up
    assert nn.bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert nn.bf16_round(-3.0) == -3.0
    x = rnd(1000)
    r = nn.bf16_round(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))  # unit roundoff of an 8-bit significand


def test_conv_matches_brute_force_loops():
    B, D, H, W, ci, co = 2, 3, 2, 4, 2, 3
    x = rnd(B, D, H, W, ci, seed=1)
    w = rnd(27, co, ci, seed=2)
    b = rnd(co, seed=3)
    y = nn.conv3d(x, w, b)
    ref = np.zeros_like(y)
    for bb in range(B):
        for z in range(D):
            for yy in range(H):
                for xx in range(W):
                    for o in range(co):
                        s = b[o]
                        t = 0
                        for dz in (-1, 0, 1):
                            for dy in (-1, 0, 1):
                                for dx in (-1, 0, 1):
                                    zz, y2, x2 = z + dz, yy + dy, xx + dx
                                    if 0 <= zz < D and 0 <= y2 < H and 0 <= x2 < W:
                                        for i in range(ci):
                                            s += w[t, o, i] * x[bb, zz, y2, x2, i]
                                    t += 1
                        ref[bb, z, yy, xx, o] = s
    np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13)


def test_conv_delta_kernels_are_identity_and_shift():
    x = rnd(1, 4, 5, 6, 3, seed=4)
    w = np.zeros((27, 3, 3))
    w[13] = np.eye(3)                         # centre tap
    np.testing.assert_array_equal(nn.conv3d(x, w), x)
    w = np.zeros((27, 3, 3))
    w[nn.TAPS.index((0, 0, 1))] = np.eye(3)   # reads x + 1
    y = nn.conv3d(x, w)
    np.testing.assert_array_equal(y[..., :-1, :], x[..., 1:, :])
    assert np.all(y[..., -1, :] == 0.0)


def test_dgrad_is_adjoint_of_conv():
    x = rnd(2, 3, 4, 5, 4, seed=5)
    w = rnd(27, 6, 4, seed=6)
    dy = rnd(2, 3, 4, 5, 6, seed=7)
    lhs = np.sum(nn.conv3d(x, w) * dy)
    rhs = np.sum(x * nn.conv3d_dgrad(dy, w))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_wgrad_bilinearity_and_finite_differences():
    x = rnd(1, 3, 4, 2, 3, seed=8)
    w = rnd(27, 2, 3, seed=9)
    b = rnd(2, seed=10)
    dy = rnd(1, 3, 4, 2, 2, seed=11)
    dw, db = nn.conv3d_wgrad(x, dy)
    lhs = np.sum(nn.conv3d(x, w) * dy)
    assert abs(lhs - np.sum(w * dw)) <= 1e-12 * abs(lhs)
    np.testing.assert_allclose(db, dy.sum(axis=(0, 1, 2, 3)))
    f = lambda ww, bb: np.sum(nn.conv3d(x, ww, bb) * dy)
    for (t, o, i) in [(0, 0, 0), (13, 1, 2), (26, 0, 1), (5, 1, 0)]:
        e = np.zeros_like(w)
        e[t, o, i] = 1e-6
        fd = (f(w + e, b) - f(w - e, b)) / 2e-6
        assert abs(fd - dw[t, o, i]) <= 1e-7 * max(1.0, abs(fd))
    e = np.zeros(2)
    e[1] = 1e-6
    assert abs((f(w, b + e) - f(w, b - e)) / 2e-6 - db[1]) < 1e-7


def test_pool_and_upsample():
    x = rnd(2, 4, 6, 2, 3, seed=12)
    y = rnd(2, 2, 3, 1, 3, seed=13)
    c = np.full((1, 4, 4, 4, 2), 2.5)
    np.testing.assert_array_equal(nn.pool2(c), np.full((1, 2, 2, 2, 2), 2.5))
    np.testing.assert_allclose(nn.pool2(nn.up2(y)), y)
    assert abs(np.sum(nn.pool2(x) * y) - np.sum(x * nn.pool2_bwd(y))) < 1e-12
    assert abs(np.sum(nn.up2(y) * x) - np.sum(y * nn.up2_bwd(x))) < 1e-12
    assert nn.up2(y)[1, 3, 5, 1, 2] == y[1, 1, 2, 0, 2]


def test_mse_gradient_finite_differences():
    y = rnd(1, 2, 2, 2, 4, seed=14)
    t = rnd(1, 2, 2, 2, 4, seed=15)
    loss, g = nn.mse(y, t, 3)
    assert abs(loss - np.mean((y[..., :3] - t[..., :3]) ** 2)) < 1e-15
    assert np.all(g[..., 3] == 0.0)
    e = np.zeros_like(y)
    e[0, 1, 0, 1, 2] = 1e-6
    fd = (nn.mse(y + e, t, 3)[0] - nn.mse(y - e, t, 3)[0]) / 2e-6
    assert abs(fd - g[0, 1, 0, 1, 2]) < 1e-8


def test_adam_first_steps_closed_form():
    w = rnd(50, seed=16)
    g = rnd(50, seed=17)
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 1e-2, 1e-8
    w1, m, v = nn.adam(w, g, m, v, 1, lr, eps=eps)
    np.testing.assert_allclose(w1, w - lr * g / (np.abs(g) + eps), rtol=1e-12)
    # the same gradient again: bias correction keeps m_hat = g, v_hat = g^2
    w2, m, v = nn.adam(w1, g, m, v, 2, lr, eps=eps)
    np.testing.assert_allclose(w2, w1 - lr * g / (np.abs(g) + eps), rtol=1e-10)


def _params(C, cin, cout, seed):
    rng = np.random.default_rng(seed)
    ps = []
    for i in range(nn.NCONV):
        ci = cin if i == 0 else C
        co = cout if i == nn.NCONV - 1 else C
        ps.append((rng.normal(size=(27, co, ci)) * np.sqrt(2.0 / (27 * ci)), rng.normal(size=co) * 0.1))
    return ps


def test_unet_gradients_finite_differences():
    C = 4
    params = _params(C, 3, 5, seed=18)
    x = rnd(1, 8, 8, 8, 3, seed=19)
    t = rnd(1, 8, 8, 8, 5, seed=20)

    def loss(ps):
        y, _ = nn.unet_forward(ps, x)
        return nn.mse(y, t, 4)[0]

    y, cache = nn.unet_forward(params, x)
    _, dy = nn.mse(y, t, 4)
    grads = nn.unet_backward(params, cache, dy)
    rng = np.random.default_rng(21)
    for i in (0, 1, 3, 6, 7, 9, 12, 14):
        w, b = params[i]
        for _ in range(2):
            idx = tuple(int(rng.integers(0, s)) for s in w.shape)
            h = 1e-6
            wp = w.copy()
            wp[idx] += h
            wm = w.copy()
            wm[idx] -= h
            pp = list(params)
            pp[i] = (wp, b)
            pm = list(params)
            pm[i] = (wm, b)
            fd = (loss(pp) - loss(pm)) / (2 * h)
            an = grads[i][0][idx]
            assert abs(fd - an) <= 1e-5 * max(abs(fd), 1e-3), (i, idx, fd, an)
        o = int(rng.integers(0, b.shape[0]))
        bp = b.copy()
        bp[o] += 1e-6
        bm = b.copy()
        bm[o] -= 1e-6
        pp = list(params)
        pp[i] = (w, bp)
        pm = list(params)
        pm[i] = (w, bm)
        fd = (loss(pp) - loss(pm)) / 2e-6
        assert abs(fd - grads[i][1][o]) <= 1e-5 * max(abs(fd), 1e-3)
