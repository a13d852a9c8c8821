"""FP64 matrix-free operator and CGLS in plain C with OpenMP (``pn_ref.c``),
for systems too large for the assembled SciPy matrix (the 128^3 P5 nebula:
76M unknowns).  ORACLE: test infrastructure only.

The row equation, the boundary rules and the solver are those of
``assemble`` / ``apply`` / ``solve`` (sections "Discretized Radiative Transfer
Equation", "Precomputation" and "Runtime"); the couplings come from
``couplings`` (quadrature) and the row diagonals from ``medium``, so the C
code only evaluates the sums.  ``tests/`` pins ``CRef.matvec`` /
``CRef.rmatvec`` to the assembled CSR matrix and ``CRef.cgls`` to SuperLU.

The shared library is compiled with gcc on first use (and whenever the C
source is newer than it).
"""
import ctypes
import os
import subprocess
import time

import numpy as np

from .assemble import cell_size
from .couplings import coupling_list
from .medium import diagonal
from .stagger import Layout

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pn_ref.c")
LIB = os.path.join(HERE, "libpnref.so")
_lib = None


def build(force=False):
    """Compiles libpnref.so (gcc, OpenMP); returns its path."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC], check=True)
        os.replace(tmp, LIB)
    return LIB


class _Op(ctypes.Structure):
    _fields_ = [("ncoeff", ctypes.c_int), ("bc", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("off", ctypes.c_void_p), ("ext", ctypes.c_void_p), ("cls", ctypes.c_void_p),
                ("ncpl", ctypes.c_int), ("ck", ctypes.c_void_p), ("cd", ctypes.c_void_p),
                ("ckp", ctypes.c_void_p), ("cv", ctypes.c_void_p), ("diag", ctypes.c_void_p)]


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        lib.ref_apply.argtypes = [ctypes.POINTER(_Op), P, P]
        lib.ref_apply_t.argtypes = [ctypes.POINTER(_Op), P, P]
        lib.ref_cgls.argtypes = [ctypes.POINTER(_Op), P, P, ctypes.c_double, ctypes.c_int, P,
                                 ctypes.POINTER(ctypes.c_double), ctypes.c_int]
        lib.ref_cgls.restype = ctypes.c_int
        lib.ref_set_threads.argtypes = [ctypes.c_int]
        lib.ref_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


class CRef:
    """FP64 operator of one medium evaluated by the C oracle."""

    def __init__(self, order, dims, sigma_t, albedo, g, sigma_t_min, bc=0, couplings=None, h=None, threads=None):
        self.lib = _load()
        if threads:
            self.lib.ref_set_threads(int(threads))
        self.threads = int(self.lib.ref_max_threads())
        lay = Layout(order, dims, bc)
        self.layout = lay
        cl = coupling_list(order) if couplings is None else couplings
        self._off = np.ascontiguousarray(lay.offset, dtype=np.int64)
        self._ext = np.ascontiguousarray(np.array(lay.ext, dtype=np.int32).reshape(-1))
        self._cls = np.ascontiguousarray(np.array(lay.cls, dtype=np.int32).reshape(-1))
        self._ck = np.array([c[0] for c in cl], dtype=np.int32)
        self._cd = np.array([c[1] for c in cl], dtype=np.int32)
        self._ckp = np.array([c[2] for c in cl], dtype=np.int32)
        self._cv = np.array([c[3] for c in cl], dtype=np.float64)
        dg = diagonal(lay, sigma_t, albedo, g, sigma_t_min)
        self._diag = np.ascontiguousarray(np.concatenate([d.reshape(-1) for d in dg]), dtype=np.float64)
        op = _Op()
        op.ncoeff = lay.ncoeff
        for d in range(3):
            op.bc[d] = int(lay.bcs[d])
        op.h = cell_size(dims, h)
        op.off, op.ext, op.cls = _ptr(self._off), _ptr(self._ext), _ptr(self._cls)
        op.ncpl = len(cl)
        op.ck, op.cd, op.ckp, op.cv = _ptr(self._ck), _ptr(self._cd), _ptr(self._ckp), _ptr(self._cv)
        op.diag = _ptr(self._diag)
        self._op = op

    @property
    def n(self):
        return self.layout.n

    def _vec(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        if x.shape != (self.n,):
            raise ValueError("vector of %d entries expected" % self.n)
        return x

    def matvec(self, x):
        x = self._vec(x)
        y = np.empty(self.n)
        self.lib.ref_apply(ctypes.byref(self._op), _ptr(x), _ptr(y))
        return y

    def rmatvec(self, x):
        x = self._vec(x)
        y = np.empty(self.n)
        self.lib.ref_apply_t(ctypes.byref(self._op), _ptr(x), _ptr(y))
        return y

    def cgls(self, b, tol, max_iter=100000, progress=0):
        """CGLS from u = 0 to ||Q - A u|| / ||Q|| <= tol (carried residual).
        Returns (u, info): iters, carried relative residual per iteration
        (history), the recomputed relative residual, seconds, threads."""
        b = self._vec(b)
        x = np.empty(self.n)
        hist = np.zeros(max_iter + 1)
        rel = ctypes.c_double(0.0)
        t0 = time.perf_counter()
        it = self.lib.ref_cgls(ctypes.byref(self._op), _ptr(b), _ptr(x), float(tol), int(max_iter), _ptr(hist),
                               ctypes.byref(rel), int(progress))
        sec = time.perf_counter() - t0
        if it < 0:
            raise MemoryError("oracle CGLS: allocation failed")
        bn = float(np.linalg.norm(b))
        true_rel = float(np.linalg.norm(b - self.matvec(x)) / bn) if bn > 0 else 0.0
        return x, dict(iters=int(it), rel_residual=true_rel, carried_rel_residual=float(rel.value),
                       history=hist[:it + 1], seconds=sec, threads=self.threads)
