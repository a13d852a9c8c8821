"""Plain FP64 reference of the learned initial guess / preconditioner network
(test infrastructure only: imported by tests and by nothing on the product
path).

The paper has no learned component; this network is the project's neural
operator that maps a medium and an isotropic source to the P3 coefficient
fields.  What it computes is defined here by its plain mathematical form:

* tensors are channels-last: x[b, z, y, x, c];
* a 3x3x3 convolution with zero padding, weights w[t, co, ci] with tap
  t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1), dz, dy, dx in {-1, 0, 1}:
      y[b, p, co] = bias[co] + sum_t sum_ci w[t, co, ci] x[b, p + d_t, ci]
  (x = 0 outside the grid);
* its input gradient is the adjoint (a scatter over taps), its weight
  gradient dw[t, co, ci] = sum_{b,p} dy[b, p, co] x[b, p + d_t, ci];
* 2x2x2 average pooling and nearest-neighbour 2x upsampling, with their
  adjoints as backward passes;
* the loss is the mean squared error over the first ``nout`` output channels;
* Adam (Kingma & Ba, "Adam: A Method for Stochastic Optimization", 2015,
  Algorithm 1) with bias correction.

A library matmul (numpy.einsum over the channel axis) serves as the channel
contraction of one tap; taps are looped explicitly.
parity of the network as a whole is pinned by finite differences and adjoint
identities, not by a published reference.
"""
import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _pad1(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))


def conv3d(x, w, bias=None):
    """y[b,p,co] = bias[co] + sum_t sum_ci w[t,co,ci] x[b,p+d_t,ci] (gather form)."""
    B, D, H, W, _ = x.shape
    xp = _pad1(np.asarray(x, dtype=np.float64))
    y = np.zeros((B, D, H, W, w.shape[1]))
    for t, (dz, dy, dx) in enumerate(TAPS):
        xs = xp[:, 1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :]
        y += np.einsum("bzyxi,oi->bzyxo", xs, w[t])
    if bias is not None:
        y += bias
    return y


def conv3d_dgrad(dy, w):
    """dx = adjoint of conv3d in x, as a scatter: dx[b, p + d_t] += w[t]^T dy[b, p]."""
    B, D, H, W, _ = dy.shape
    dxp = np.zeros((B, D + 2, H + 2, W + 2, w.shape[2]))
    for t, (dz, dy_, dx) in enumerate(TAPS):
        dxp[:, 1 + dz:1 + dz + D, 1 + dy_:1 + dy_ + H, 1 + dx:1 + dx + W, :] += np.einsum("bzyxo,oi->bzyxi", dy, w[t])
    return dxp[:, 1:-1, 1:-1, 1:-1, :]


def conv3d_wgrad(x, dy):
    """(dw, dbias): dw[t,co,ci] = sum_{b,p} dy[b,p,co] x[b,p+d_t,ci]; dbias = sum dy."""
    B, D, H, W, _ = x.shape
    xp = _pad1(np.asarray(x, dtype=np.float64))
    dw = np.zeros((27, dy.shape[-1], x.shape[-1]))
    for t, (dz, dy_, dx) in enumerate(TAPS):
        xs = xp[:, 1 + dz:1 + dz + D, 1 + dy_:1 + dy_ + H, 1 + dx:1 + dx + W, :]
        dw[t] = np.einsum("bzyxo,bzyxi->oi", dy, xs)
    return dw, dy.sum(axis=(0, 1, 2, 3))


def pool2(x):
    """2x2x2 average pooling (even extents)."""
    B, D, H, W, C = x.shape
    return x.reshape(B, D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4, 6))


def pool2_bwd(dy):
    """Adjoint of pool2: every fine cell receives 1/8 of its coarse gradient."""
    return np.repeat(np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up2(x):
    """Nearest-neighbour 2x upsampling."""
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up2_bwd(dy):
    """Adjoint of up2: the sum over each 2x2x2 block."""
    B, D, H, W, C = dy.shape
    return dy.reshape(B, D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4, 6))


def mse(y, t, nout):
    """(loss, dloss/dy): mean over voxels and the first nout channels."""
    diff = np.zeros_like(y)
    diff[..., :nout] = y[..., :nout] - t[..., :nout]
    cnt = y[..., :nout].size
    return float((diff ** 2).sum() / cnt), 2.0 * diff / cnt


def adam(w, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------------- U-Net --
# 4 levels, C channels everywhere; conv index -> (level, role):
#   0,1 encoder level 0 | 2,3 level 1 | 4,5 level 2 | 6,7 bottleneck (level 3)
#   8,9 decoder level 2 | 10,11 level 1 | 12,13 level 0 | 14 output (no ReLU)
NCONV = 15


def unet_forward(params, x, quant=False):
    """Forward pass; returns (output, cache).  params: list of (w, b).
    quant=True rounds every stored activation to bfloat16, as the device
    network stores them."""
    q = bf16_round if quant else (lambda a: a)
    cache = {"x": x}

    def cr(i, h):  # conv + bias + ReLU
        pre = conv3d(h, *params[i])
        cache["in%d" % i] = h
        out = q(np.maximum(pre, 0.0))
        cache["out%d" % i] = out
        return out

    h = cr(1, cr(0, x))
    s0 = h
    h = cr(3, cr(2, q(pool2(h))))
    s1 = h
    h = cr(5, cr(4, q(pool2(h))))
    s2 = h
    h = cr(7, cr(6, q(pool2(h))))
    h = cr(9, cr(8, q(up2(h) + s2)))
    h = cr(11, cr(10, q(up2(h) + s1)))
    h = cr(13, cr(12, q(up2(h) + s0)))
    cache["in14"] = h
    y = conv3d(h, *params[14])
    return y, cache


def unet_backward(params, cache, dy):
    """Gradients (dw, db) of every conv for the output gradient dy."""
    grads = [None] * NCONV

    def conv_back(i, g, relu=True):
        if relu:
            g = g * (cache["out%d" % i] > 0.0)
        grads[i] = conv3d_wgrad(cache["in%d" % i], g)
        return conv3d_dgrad(g, params[i][0])

    g = conv_back(14, dy, relu=False)
    g = conv_back(12, conv_back(13, g))
    gs0 = g                      # the skip receives the sum's gradient
    g = up2_bwd(g)
    g = conv_back(10, conv_back(11, g))
    gs1 = g
    g = up2_bwd(g)
    g = conv_back(8, conv_back(9, g))
    gs2 = g
    g = up2_bwd(g)
    g = conv_back(6, conv_back(7, g))
    g = pool2_bwd(g) + gs2
    g = conv_back(4, conv_back(5, g))
    g = pool2_bwd(g) + gs1
    g = conv_back(2, conv_back(3, g))
    g = pool2_bwd(g) + gs0
    conv_back(0, conv_back(1, g))
    return grads
