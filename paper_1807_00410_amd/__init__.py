"""MI355X-native staggered-grid real P_N solver (HIP kernels behind a C ABI).

The compute path is libpn.so (built from csrc/ by ``build.py``); this package
only marshals torch device tensors into the C ABI of include/pn.h.  There is
no CPU fallback: loading fails loudly when the library is missing.
"""
from . import _lib  # noqa: F401


def __getattr__(name):
    if name in ("Solver", "PnError", "Layout", "coupling_table"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
