"""Matrix-free FP64 apply of A and A^T (oracle; test infrastructure only).

Same rows as ``assemble`` (the real P_N equations discretised by central
differences on the staggered grid), evaluated with whole-array NumPy slices so
that grids too large for an assembled matrix can be checked.  ``A^T`` is the
literal transpose: every entry (row, col, v) of A is scattered as (col, row, v).
It does not use the skew symmetry of the transport part; ``tests/`` checks
that property separately.  Boundary rules per axis as in ``assemble``
(dropped, wrapped, or moved to the closest index inside for Neumann).

``tests/`` pins both functions, and ``rows_of``, to the CSR matrix of
``assemble`` on small grids.
"""
import numpy as np

from .assemble import cell_size
from .couplings import coupling_list
from .medium import diagonal
from .stagger import Layout, BC_PERIODIC, BC_NEUMANN, resolve_index

_AXIS = (2, 1, 0)  # x, y, z -> axis of an (ez, ey, ex) array


def _gather(arr, d, offset, out_len, bc):
    """b[i] = arr[i + offset] along axis d for i < out_len; 0 outside (vacuum),
    wrapped (periodic) or the closest entry inside (Neumann)."""
    ax = _AXIS[d]
    n = arr.shape[ax]
    idx = np.arange(out_len) + offset
    if bc == BC_PERIODIC:
        return np.take(arr, np.mod(idx, n), axis=ax)
    if bc == BC_NEUMANN:
        return np.take(arr, np.clip(idx, 0, n - 1), axis=ax)
    keep = (idx >= 0) & (idx < n)
    shape = list(arr.shape)
    shape[ax] = out_len
    out = np.zeros(shape)
    sl_out = [slice(None)] * 3
    sl_out[ax] = np.nonzero(keep)[0]
    out[tuple(sl_out)] = np.take(arr, idx[keep], axis=ax)
    return out


def _scatter_add(dst, src, d, offset, bc):
    """dst[i + offset] += src[i] along axis d (dropped outside under the
    vacuum boundary, wrapped if periodic, clamped inside under Neumann)."""
    ax = _AXIS[d]
    n = dst.shape[ax]
    idx = np.arange(src.shape[ax]) + offset
    if bc == BC_PERIODIC:
        idx = np.mod(idx, n)
        keep = np.ones(idx.shape, dtype=bool)
    elif bc == BC_NEUMANN:
        idx = np.clip(idx, 0, n - 1)
        keep = np.ones(idx.shape, dtype=bool)
    else:
        keep = (idx >= 0) & (idx < n)
    for j in np.nonzero(keep)[0]:
        sl_d = [slice(None)] * 3
        sl_s = [slice(None)] * 3
        sl_d[ax] = idx[j]
        sl_s[ax] = j
        dst[tuple(sl_d)] += src[tuple(sl_s)]


class Operator:
    """FP64 matrix-free operator of one medium."""

    def __init__(self, order, dims, sigma_t, albedo, g, sigma_t_min, bc=0, couplings=None, h=None):
        self.layout = Layout(order, dims, bc)
        self.couplings = coupling_list(order) if couplings is None else couplings
        self.diag = diagonal(self.layout, sigma_t, albedo, g, sigma_t_min)
        self.h = cell_size(dims, h)
        self.bcs = self.layout.bcs

    @property
    def n(self):
        return self.layout.n

    def matvec(self, x):
        lay = self.layout
        x = np.asarray(x, dtype=np.float64)
        y = np.zeros(lay.n)
        for k in range(lay.ncoeff):
            lay.view(y, k)[...] = self.diag[k] * lay.view(x, k)
        for (k, d, kp, c) in self.couplings:
            xk = lay.view(x, kp)
            out_len = lay.ext[k][d]
            if lay.cls[kp][d] == 1:
                plus, minus = _gather(xk, d, 1, out_len, self.bcs[d]), _gather(xk, d, 0, out_len, self.bcs[d])
            else:
                plus, minus = _gather(xk, d, 0, out_len, self.bcs[d]), _gather(xk, d, -1, out_len, self.bcs[d])
            lay.view(y, k)[...] += (c / self.h) * (plus - minus)
        return y

    def rmatvec(self, x):
        lay = self.layout
        x = np.asarray(x, dtype=np.float64)
        y = np.zeros(lay.n)
        for k in range(lay.ncoeff):
            lay.view(y, k)[...] = self.diag[k] * lay.view(x, k)
        for (k, d, kp, c) in self.couplings:
            src = (c / self.h) * lay.view(x, k)
            dst = lay.view(y, kp)
            b = self.bcs[d]
            if lay.cls[kp][d] == 1:
                _scatter_add(dst, src, d, 1, b)
                _scatter_add(dst, -src, d, 0, b)
            else:
                _scatter_add(dst, src, d, 0, b)
                _scatter_add(dst, -src, d, -1, b)
        return y


def rows_of(order, dims, sigma_t, albedo, g, sigma_t_min, x, rows, bc=0, couplings=None, absolute=False,
            h=None):
    """(A x)[row] for the given flat row indices, evaluated one row at a time
    from the row equation (no assembled matrix, no whole-grid arrays).  For
    spot checks of grids too large for ``Operator``.  With ``absolute=True``
    returns (|A| |x|)[row] instead: every term of the row taken in magnitude,
    the collision and scattering parts of the diagonal separately
    (sigma_t + |g|^l sigma_s), the scale of a rounding-error bound."""
    ab = abs if absolute else (lambda v: v)
    from .sh import coeff_lm
    lay = Layout(order, dims, bc)
    bcs = lay.bcs
    cl = coupling_list(order) if couplings is None else couplings
    by_row = {}
    for (k, d, kp, c) in cl:
        by_row.setdefault(k, []).append((d, kp, c))
    st = np.maximum(np.asarray(sigma_t, dtype=np.float64), float(np.float32(sigma_t_min)))
    ss = np.asarray(albedo, dtype=np.float64) * st
    n = (dims[0], dims[1], dims[2])
    h = cell_size(dims, h)
    g = float(np.float32(g))
    x = np.asarray(x)
    out = np.empty(len(rows))
    for t, row in enumerate(rows):
        k = int(np.searchsorted(lay.offset, row, side="right") - 1)
        ex, ey, ez = lay.ext[k]
        loc = int(row - lay.offset[k])
        pt = [loc % ex, (loc // ex) % ey, loc // (ex * ey)]
        p = lay.cls[k]
        # parameters: mean over the adjacent cells (clamped or wrapped), z-major order
        cand = []
        for d in range(3):
            cs = [pt[d]] if p[d] == 0 else [pt[d] - 1, pt[d]]
            cand.append([(c % n[d]) if bcs[d] == BC_PERIODIC else min(max(c, 0), n[d] - 1) for c in cs])
        tsum, ssum, cnt = 0.0, 0.0, 0
        for cz in cand[2]:
            for cy in cand[1]:
                for cx in cand[0]:
                    tsum += st[cz, cy, cx]
                    ssum += ss[cz, cy, cx]
                    cnt += 1
        l = coeff_lm(k)[0]
        if absolute:  # magnitudes before the sigma_t - g^l sigma_s cancellation
            val = (tsum / cnt + (abs(float(g)) ** l) * (ssum / cnt)) * abs(float(x[row]))
        else:
            val = (tsum / cnt - (float(g) ** l) * (ssum / cnt)) * float(x[row])
        for (d, kp, c) in by_row.get(k, []):
            pe = lay.ext[kp]
            i = pt[d]
            ip, im = (i + 1, i) if lay.cls[kp][d] == 1 else (i, i - 1)
            for idx, sgn in ((ip, 1.0), (im, -1.0)):
                idx = resolve_index(idx, pe[d], bcs[d])
                if idx is None:
                    continue
                q = list(pt)
                q[d] = idx
                col = lay.offset[kp] + (q[2] * pe[1] + q[1]) * pe[0] + q[0]
                val += ab(sgn * c / h * float(x[col]))
        out[t] = val
    return out
