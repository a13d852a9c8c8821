"""FP64 reference of the multigrid preconditioner of the even-parity PCG, for
the GPU tests (test infrastructure; shares nothing with the library).

The preconditioner is this library's own design, not the paper's (the paper
names multigrid only as future work), so this is its definition written out
with sparse matrices from the oracle's assembled system:

* S = D_e + T_eo D_o^-1 T_eo^T, the Schur complement of the even bands
  (assembled from the oracle's matrix A = [[D_e, T_eo], [-T_eo^T, D_o]]);
  S_k its diagonal block for the even coefficient k, with the couplings
  across a periodic seam removed from the off-diagonal (they stay on the
  diagonal): C_k.
* P_L: piecewise-constant prolongation over 2 x 2 x 2 aggregates of a
  lattice of extents e to one of ceil(e / 2); levels are added until every
  slot's extents are at most 5 and all slots together hold at most 2048
  points (at most 11 coarse levels).  A_1 = P_0^T C_k P_0, A_{L+1} =
  P_L^T A_L P_L.
* V on level L: z = w D^-1 r (w = 0.9); r_c = P_L^T (r - A z); z += P_L
  V(r_c); z += w D^-1 (r - A z).  On the coarsest level: 16 damped Jacobi
  sweeps from zero.
* B r = 0.6 M r + P_0 V(P_0^T r) on the even entries, 0 on the odd ones, M
  the Jacobi inverse diagonal (taken here from the library's Jacobi
  preconditioner, which another test pins to 1 / diag(S)).
"""
import numpy as np
import scipy.sparse as sp

from oracle.sh import coeff_lm

OMEGA = 0.9
OMEGA_FINE = 0.6
SWEEPS = 16
COARSEST_EXT = 5
COARSEST_MAX = 2048
MAX_LEVELS = 12


def schur_even(A, lay):
    """(S, E): the even-band Schur complement and the global indices of its rows."""
    A = A.tocsr()
    par = np.concatenate([np.full(lay.size[k], coeff_lm(k)[0] % 2) for k in range(lay.ncoeff)])
    E, O = np.nonzero(par == 0)[0], np.nonzero(par == 1)[0]
    S = sp.diags(A[E][:, E].diagonal()) - A[E][:, O] @ sp.diags(1.0 / A[O][:, O].diagonal()) @ A[O][:, E]
    return S.tocsr(), E


def coords(ext):
    ex, ey, ez = ext
    z, y, x = np.meshgrid(np.arange(ez), np.arange(ey), np.arange(ex), indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def prolongation(ext):
    """P (fine points x coarse points), both lattices numbered x fastest."""
    cx, cy, cz = [(e + 1) // 2 for e in ext]
    x, y, z = coords(ext)
    coarse = ((z // 2) * cy + (y // 2)) * cx + (x // 2)
    nf = ext[0] * ext[1] * ext[2]
    return sp.csr_matrix((np.ones(nf), (np.arange(nf), coarse)), shape=(nf, cx * cy * cz)), (cx, cy, cz)


def level_extents(exts):
    """Per level (from 0) the list of the slots' extents."""
    geo = [list(exts)]
    while True:
        nxt = [tuple((e + 1) // 2 for e in ext) for ext in geo[-1]]
        geo.append(nxt)
        mx = max(max(e) for e in nxt)
        tot = sum(e[0] * e[1] * e[2] for e in nxt)
        if (mx <= COARSEST_EXT and tot <= COARSEST_MAX) or len(geo) >= MAX_LEVELS:
            return geo


def cut_seams(Sk, ext):
    """Off-diagonal entries of Sk between points more than one lattice step
    apart along some axis (periodic wrap-around) removed."""
    C = Sk.tocoo()
    x, y, z = coords(ext)
    far = ((np.abs(x[C.row] - x[C.col]) > 1) | (np.abs(y[C.row] - y[C.col]) > 1)
           | (np.abs(z[C.row] - z[C.col]) > 1))
    keep = ~far | (C.row == C.col)
    return sp.csr_matrix((C.data[keep], (C.row[keep], C.col[keep])), shape=C.shape)


def vcycle(As, Ps, L, r):
    A = As[L]
    d = A.diagonal()
    if L == len(As) - 1:
        z = np.zeros_like(r)
        for _ in range(SWEEPS):
            z = z + OMEGA * (r - A @ z) / d
        return z
    z = OMEGA * r / d
    rc = Ps[L].T @ (r - A @ z)
    z = z + Ps[L] @ vcycle(As, Ps, L + 1, rc)
    return z + OMEGA * (r - A @ z) / d


def apply_mg(A, lay, r, z_jacobi):
    """B r (length lay.n, FP64) for the packed residual r and the library's
    Jacobi preconditioner output z_jacobi = M r."""
    S, E = schur_even(A, lay)
    pos = np.full(lay.n, -1, dtype=np.int64)
    pos[E] = np.arange(E.size)
    even = [k for k in range(lay.ncoeff) if coeff_lm(k)[0] % 2 == 0]
    geo = level_extents([lay.ext[k] for k in even])
    out = np.zeros(lay.n)
    r = np.asarray(r, dtype=np.float64)
    for s, k in enumerate(even):
        idx = np.arange(lay.offset[k], lay.offset[k + 1])
        ek = pos[idx]
        Sk = S[ek][:, ek]
        Ps = []
        As = [cut_seams(Sk, geo[0][s])]
        for L in range(len(geo) - 1):
            P, _ = prolongation(geo[L][s])
            Ps.append(P)
            As.append((P.T @ As[-1] @ P).tocsr())
        # level 0 carries only the prolongation: the V-cycle starts on level 1
        z1 = vcycle(As[1:], Ps[1:], 0, Ps[0].T @ r[idx])
        out[idx] = OMEGA_FINE * np.asarray(z_jacobi, dtype=np.float64)[idx] + Ps[0] @ z1
    return out
