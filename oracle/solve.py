"""Solvers for A u = Q in FP64 (oracle; test infrastructure only).

* ``direct``: sparse LU (SciPy SuperLU) of the assembled matrix -- the exact
  solution up to rounding, for tiny grids.
* ``cgls``: the paper's solver (section "Runtime" and "Results"): conjugate
  gradients on the normal equations A^T A u = A^T Q without forming A^T A
  (A is non-symmetric and not diagonally dominant).  Written in the usual
  CGLS form, with the residual r = Q - A u carried along; the stopping test is
  the relative residual of the original system ||Q - A u|| / ||Q||, and the
  returned residual is recomputed from scratch.
"""
import time

import numpy as np
import scipy.sparse.linalg as spla


def direct(A, b):
    """u = A^{-1} b by SuperLU."""
    lu = spla.splu(A.tocsc())
    return lu.solve(np.asarray(b, dtype=np.float64))


def rel_residual(matvec, u, b):
    r = np.asarray(b, dtype=np.float64) - matvec(u)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def cgls(matvec, rmatvec, b, tol=1e-10, max_iter=100000, x0=None, callback=None):
    """CGLS for min ||b - A x||.  Returns (x, info) with info = dict(iters,
    rel_residual (recomputed), history (recursive residuals), seconds)."""
    t0 = time.perf_counter()
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    if bnorm == 0.0:
        return np.zeros_like(b), dict(iters=0, rel_residual=0.0, history=[0.0], seconds=0.0)
    r = b - matvec(x) if x0 is not None else b.copy()
    s = rmatvec(r)
    p = s.copy()
    gamma = float(s @ s)
    hist = [float(np.linalg.norm(r)) / bnorm]
    it = 0
    while hist[-1] > tol and it < max_iter and gamma > 0.0:
        q = matvec(p)
        alpha = gamma / float(q @ q)
        x += alpha * p
        r -= alpha * q
        s = rmatvec(r)
        gamma_new = float(s @ s)
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
        it += 1
        hist.append(float(np.linalg.norm(r)) / bnorm)
        if callback is not None:
            callback(it, hist[-1])
    return x, dict(iters=it, rel_residual=rel_residual(matvec, x, b), history=hist,
                   seconds=time.perf_counter() - t0)
