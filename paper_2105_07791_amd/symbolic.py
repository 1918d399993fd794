"""Host-only access to the library's symbolic analysis (no GPU needed)."""
import ctypes as C

import numpy as np

from . import _lib
from ._lib import check, lib

__all__ = ["Analysis", "read_tree", "read_perm"]


def read_perm(handle, n):
    p = np.empty(n, dtype=np.int32)
    check(lib().hssx_get_perm(handle, p.ctypes.data_as(_lib._ip), n))
    return p


def read_tree(handle):
    """Flattened elimination and cluster trees of a factor/analysis handle."""
    sz = np.zeros(4, dtype=np.int64)
    check(lib().hssx_get_tree(handle, sz.ctypes.data_as(_lib._i64p),
                              None, None, None, None, None, None, None))
    nn, ti, tb, tc = (int(v) for v in sz)
    a = lambda k: np.empty(k, dtype=np.int32)
    info, iid, iptr, bid, bptr, cl, cptr = a(10 * nn), a(ti), a(nn + 1), a(tb), a(nn + 1), \
        a(5 * tc), a(nn + 1)
    P = lambda v: v.ctypes.data_as(_lib._ip)
    check(lib().hssx_get_tree(handle, sz.ctypes.data_as(_lib._i64p), P(info), P(iid),
                              P(iptr), P(bid), P(bptr), P(cl), P(cptr)))
    return dict(info=info.reshape(nn, 10), I=iid, I_ptr=iptr, B=bid, B_ptr=bptr,
                clusters=cl.reshape(tc, 5), c_ptr=cptr)


class Analysis:
    """Symbolic analysis of an N x N grid with `dofs` unknowns per node
    (hssx_analyze), or with dg=True of the N x N x 2 triangle mesh of the
    SIPG operator of degree p (hssx_analyze_ipdg; 6 DOFs per triangle for
    p = 2, 3 for p = 1)."""

    def __init__(self, N, leaf_size=32, beta=16, dofs=1, dg=False, p=2):
        h = C.c_void_p()
        if dg:
            nb = 3 if p == 1 else 6
            self.N, self.n, self.dofs = N, 2 * nb * N * N, nb
            check(lib().hssx_analyze_ipdg(int(N), int(p), int(leaf_size), int(beta), C.byref(h)))
        else:
            self.N, self.n, self.dofs = N, N * N * dofs, dofs
            check(lib().hssx_analyze(int(N), int(dofs), int(leaf_size), int(beta), C.byref(h)))
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and getattr(_lib, "_LIB", None) is not None:
            lib().hssx_fact_destroy(self.handle)
            self.handle = None

    def perm(self):
        return read_perm(self.handle, self.n)

    def tree(self):
        return read_tree(self.handle)
