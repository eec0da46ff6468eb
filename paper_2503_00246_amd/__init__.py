"""MI355X-native matrix-free ghost-penalty operator y = G(gamma) u.

The compute path is the HIP library libghost.so (C ABI declared in
include/ghost.h); this package is a thin ctypes binding over it plus an
autograd wrapper.  The library is loaded on first use and its absence is an
error: there is no CPU fallback.
"""

__all__ = ["GhostOperator", "GhostApply", "ghost_apply", "cg_solve"]


def __getattr__(name):
    if name in ("GhostOperator", "cg_solve"):
        from . import operator as _op
        return getattr(_op, name)
    if name in ("GhostApply", "ghost_apply"):
        from . import autograd as _ag
        return getattr(_ag, name)
    raise AttributeError(name)
