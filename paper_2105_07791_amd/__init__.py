"""MI355X-native hierarchical nested-dissection + HSS preconditioner for 2D
Galerkin wave problems (Bonev & Hesthaven).  The computation lives in
libhssx.so (HIP, gfx950); this package only marshals arguments."""
from ._lib import HssxError, lib  # noqa: F401


def __getattr__(name):
    # the torch-facing binding is imported lazily so that the C-ABI loader
    # can be checked without initialising a GPU
    if name in ("Operator", "BatchOperator", "Factor", "assemble", "factor", "gmres_solve"):
        from . import hssx
        return getattr(hssx, name)
    if name in ("WaveSolve",):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
