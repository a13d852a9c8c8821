"""Python handle around the network ABI (include/pn_nn.h): argument
marshalling of torch device tensors; every layer runs in the HIP library.

Activations are torch.bfloat16 tensors of shape [B, nz, ny, nx, 32]
(channels-last), convolution weights torch.bfloat16 [27, 32, 32] (tap, out,
in)."""
import ctypes as C

import torch

from . import _lib as L

KC = 32


class NetError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d): %s" % (L.load().pn_status_string(status).decode(), status, msg))
        self.status = status


def _p(t, dtype=None):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError("expected %s, got %s" % (dtype, t.dtype))
    return C.c_void_p(t.data_ptr())


def _s(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _chk(rc):
    if rc != L.PN_OK:
        raise NetError(rc, L.load().pn_nn_last_error().decode())


def _dims(x):
    B, nz, ny, nx, c = x.shape
    if c != KC:
        raise ValueError("expected %d channels" % KC)
    return B, nx, ny, nz


def conv3d(x, w, bias=None, relu=False, out_f32=False, stream=None):
    B, nx, ny, nz = _dims(x)
    y = torch.empty(x.shape, dtype=torch.float32 if out_f32 else torch.bfloat16, device=x.device)
    _chk(L.load().pn_nn_conv3d(B, nx, ny, nz, _p(x, torch.bfloat16), _p(w, torch.bfloat16),
                               _p(bias, torch.float32), int(relu), int(out_f32), _p(y), _s(stream)))
    return y


def conv3d_dgrad(g, w, stream=None):
    B, nx, ny, nz = _dims(g)
    dx = torch.empty_like(g)
    _chk(L.load().pn_nn_conv3d_dgrad(B, nx, ny, nz, _p(g, torch.bfloat16), _p(w, torch.bfloat16), _p(dx),
                                     _s(stream)))
    return dx


def conv3d_wgrad(x, g, stream=None):
    B, nx, ny, nz = _dims(x)
    dw = torch.empty((27, KC, KC), dtype=torch.float32, device=x.device)
    db = torch.empty(KC, dtype=torch.float32, device=x.device)
    _chk(L.load().pn_nn_conv3d_wgrad(B, nx, ny, nz, _p(x, torch.bfloat16), _p(g, torch.bfloat16), _p(dw), _p(db),
                                     _s(stream)))
    return dw, db


def conv3d_wgrad_noalloc(x, g, dw, db, stream=None):
    """Weight gradient into caller-provided dw (FP32 [27, 32, 32]) and db
    (FP32 [32]) through the allocation-free entry point (asynchronous)."""
    B, nx, ny, nz = _dims(x)
    if dw.shape != (27, KC, KC) or db.shape != (KC,):
        raise ValueError("dw must be [27, 32, 32] and db [32]")
    _chk(L.load().pn_nn_conv3d_wgrad_noalloc(B, nx, ny, nz, _p(x, torch.bfloat16), _p(g, torch.bfloat16),
                                             _p(dw, torch.float32), _p(db, torch.float32), _s(stream)))
    return dw, db


def pool2(x, stream=None):
    B, nx, ny, nz = _dims(x)
    y = torch.empty((B, nz // 2, ny // 2, nx // 2, KC), dtype=torch.bfloat16, device=x.device)
    _chk(L.load().pn_nn_pool2(B, nx, ny, nz, _p(x, torch.bfloat16), _p(y), _s(stream)))
    return y


def pool2_bwd_add(gc, skip=None, stream=None):
    B, nx, ny, nz = _dims(gc)
    gf = torch.empty((B, 2 * nz, 2 * ny, 2 * nx, KC), dtype=torch.bfloat16, device=gc.device)
    _chk(L.load().pn_nn_pool2_bwd_add(B, 2 * nx, 2 * ny, 2 * nz, _p(gc, torch.bfloat16), _p(skip, torch.bfloat16),
                                      _p(gf), _s(stream)))
    return gf


def up2_add(xc, skip=None, stream=None):
    B, nx, ny, nz = _dims(xc)
    y = torch.empty((B, 2 * nz, 2 * ny, 2 * nx, KC), dtype=torch.bfloat16, device=xc.device)
    _chk(L.load().pn_nn_up2_add(B, 2 * nx, 2 * ny, 2 * nz, _p(xc, torch.bfloat16), _p(skip, torch.bfloat16),
                                _p(y), _s(stream)))
    return y


def up2_bwd(gf, stream=None):
    B, nx, ny, nz = _dims(gf)
    gc = torch.empty((B, nz // 2, ny // 2, nx // 2, KC), dtype=torch.bfloat16, device=gf.device)
    _chk(L.load().pn_nn_up2_bwd(B, nx, ny, nz, _p(gf, torch.bfloat16), _p(gc), _s(stream)))
    return gc


def adam(w, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _chk(L.load().pn_nn_adam(_p(w, torch.float32), _p(g, torch.float32), _p(m, torch.float32),
                             _p(v, torch.float32), w.numel(), int(step), float(lr), float(beta1), float(beta2),
                             float(eps), _s(stream)))


class Net:
    """The 4-level U-Net (pn_net_*)."""

    def __init__(self, seed=0, stream=None):
        self.lib = L.load()
        n = C.c_void_p()
        rc = self.lib.pn_net_create(int(seed), _s(stream), C.byref(n))
        if rc != L.PN_OK:
            raise NetError(rc, self.lib.pn_net_last_error(None).decode())
        self.n = n
        self.nparams = self.lib.pn_net_nparams()

    def _check(self, rc):
        if rc != L.PN_OK:
            raise NetError(rc, self.lib.pn_net_last_error(self.n).decode())

    def close(self):
        if getattr(self, "n", None):
            self.lib.pn_net_destroy(self.n)
            self.n = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        import numpy as np
        p = np.empty(self.nparams, dtype=np.float32)
        self._check(self.lib.pn_net_get_params(self.n, p.ctypes.data_as(C.c_void_p), None))
        return p

    def grads(self):
        import numpy as np
        g = np.empty(self.nparams, dtype=np.float32)
        self._check(self.lib.pn_net_get_params(self.n, None, g.ctypes.data_as(C.c_void_p)))
        return g

    def set_params(self, p):
        import numpy as np
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.nparams
        self._check(self.lib.pn_net_set_params(self.n, p.ctypes.data_as(C.c_void_p)))

    def save(self, path):
        self._check(self.lib.pn_net_save(self.n, str(path).encode()))

    def load(self, path):
        self._check(self.lib.pn_net_load(self.n, str(path).encode()))

    def forward(self, x):
        B, nx, ny, nz = _dims(x)
        y = torch.empty(x.shape, dtype=torch.float32, device=x.device)
        self._check(self.lib.pn_net_forward(self.n, B, nx, ny, nz, _p(x, torch.bfloat16), _p(y)))
        return y

    def train(self, xs, ts, epochs, batch, lr, seed=0):
        """pn_net_train over lists of per-sample tensors x [1, nz, ny, nx, 32]
        and target [1, nz, ny, nx, nout]; returns the last epoch's mean loss."""
        _, nx, ny, nz = _dims(xs[0])
        xp = (C.c_void_p * len(xs))(*[_p(v, torch.bfloat16).value for v in xs])
        tp = (C.c_void_p * len(ts))(*[_p(v, torch.bfloat16).value for v in ts])
        loss = C.c_double()
        self._check(self.lib.pn_net_train(self.n, len(xs), nx, ny, nz, xp, tp, int(ts[0].shape[-1]), int(epochs),
                                          int(batch), float(lr), int(seed), C.byref(loss)))
        return loss.value

    def train_step(self, x, target, lr):
        B, nx, ny, nz = _dims(x)
        loss = C.c_double()
        self._check(self.lib.pn_net_train_step(self.n, B, nx, ny, nz, _p(x, torch.bfloat16),
                                               _p(target, torch.bfloat16), int(target.shape[-1]), float(lr),
                                               C.byref(loss)))
        return loss.value
