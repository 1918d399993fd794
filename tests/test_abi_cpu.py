"""C-ABI library checks that need no GPU: every symbol declared in
include/hssx.h is exported, and the library's host symbolic analysis equals
the oracle's bit for bit (integer index work, Sec. 3.1-3.3)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import nd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2105_07791_amd", "libhssx.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhssx.so not built")


def _declared():
    text = open(os.path.join(ROOT, "include", "hssx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hssx_[a-zA-Z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 15
    L = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("N,leaf,beta,dofs", [(9, 8, 4, 1), (17, 32, 16, 1), (40, 20, 8, 1),
                                              (65, 32, 16, 1), (100, 32, 16, 1),
                                              (129, 24, 12, 1), (513, 32, 16, 1),
                                              (9, 8, 4, 2), (33, 33, 17, 2), (64, 32, 16, 2),
                                              (101, 48, 24, 2)])
def test_symbolic_bit_exact(N, leaf, beta, dofs):
    from paper_2105_07791_amd.symbolic import Analysis
    an = Analysis(N, leaf, beta, dofs=dofs)
    t = nd.build_nd(N, leaf, beta, dofs=dofs)
    assert np.array_equal(an.perm(), t.perm)
    tr = an.tree()
    assert tr["info"].shape[0] == len(t.boxes)
    for k, b in enumerate(t.boxes):
        info = tr["info"][k]
        assert list(info) == [b.x0, b.x1, b.y0, b.y1, b.lo, b.hi, b.parent, b.depth,
                              b.height, b.p0], k
        assert np.array_equal(tr["I"][tr["I_ptr"][k]:tr["I_ptr"][k + 1]], b.I), k
        assert np.array_equal(tr["B"][tr["B_ptr"][k]:tr["B_ptr"][k + 1]], b.B), k
        cl = tr["clusters"][tr["c_ptr"][k]:tr["c_ptr"][k + 1]]
        ct = b.ctree
        ref = np.stack([ct.start, ct.size, ct.left, ct.right, ct.level], axis=1) \
            if ct.nclusters else np.zeros((0, 5))
        assert np.array_equal(cl, ref), k


@pytest.mark.parametrize("Nc,leaf,beta,p", [(1, 12, 6, 2), (3, 12, 12, 2), (8, 60, 60, 2),
                                            (11, 36, 24, 2), (32, 60, 60, 2), (45, 60, 30, 2),
                                            (2, 6, 3, 1), (9, 30, 30, 1), (22, 30, 30, 1),
                                            (45, 30, 30, 1)])
def test_symbolic_dg_bit_exact(Nc, leaf, beta, p):
    from paper_2105_07791_amd.symbolic import Analysis
    an = Analysis(Nc, leaf, beta, dg=True, p=p)
    t = nd.build_nd_dg(Nc, leaf, beta, dofs=3 if p == 1 else 6)
    assert np.array_equal(an.perm(), t.perm)
    tr = an.tree()
    assert tr["info"].shape[0] == len(t.boxes)
    for k, b in enumerate(t.boxes):
        info = tr["info"][k]
        assert list(info) == [b.x0, b.x1, b.y0, b.y1, b.lo, b.hi, b.parent, b.depth,
                              b.height, b.p0], k
        assert np.array_equal(tr["I"][tr["I_ptr"][k]:tr["I_ptr"][k + 1]], b.I), k
        assert np.array_equal(tr["B"][tr["B_ptr"][k]:tr["B_ptr"][k + 1]], b.B), k
        cl = tr["clusters"][tr["c_ptr"][k]:tr["c_ptr"][k + 1]]
        ct = b.ctree
        ref = np.stack([ct.start, ct.size, ct.left, ct.right, ct.level], axis=1) \
            if ct.nclusters else np.zeros((0, 5))
        assert np.array_equal(cl, ref), k


def test_invalid_arguments_rejected():
    from paper_2105_07791_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.hssx_analyze(1, 1, 32, 16, ctypes.byref(h)) == -1
    assert b"invalid" in L.hssx_last_error()
    assert L.hssx_analyze(9, 1, 0, 16, ctypes.byref(h)) == -1
    assert L.hssx_analyze(9, 2, 1, 16, ctypes.byref(h)) == -1
    assert L.hssx_analyze(9, 3, 32, 16, ctypes.byref(h)) == -1
    assert L.hssx_analyze_dg(0, 60, 60, ctypes.byref(h)) == -1
    assert L.hssx_analyze_dg(8, 5, 60, ctypes.byref(h)) == -1
    assert L.hssx_analyze_ipdg(8, 3, 30, 30, ctypes.byref(h)) == -1
    assert L.hssx_analyze_ipdg(8, 1, 2, 30, ctypes.byref(h)) == -1
    # IPDG assembly arguments are checked before any device call
    bad = [_lib.IpdgDesc(8, 3, _lib.BC_DIRICHLET, 1.0), _lib.IpdgDesc(8, 1, 7, 1.0),
           _lib.IpdgDesc(0, 1, _lib.BC_DIRICHLET, 1.0), _lib.IpdgDesc(5401, 1, _lib.BC_DIRICHLET, 1.0),
           _lib.IpdgDesc(8, 1, _lib.BC_DIRICHLET, -1.0)]
    for d in bad:
        assert L.hssx_assemble_ipdg(0, ctypes.byref(d), ctypes.c_void_p(8), None,
                                    ctypes.byref(h)) == -1
    assert L.hssx_assemble_ipdg(0, None, ctypes.c_void_p(8), None, ctypes.byref(h)) == -1
    # HSS building blocks: op range, and the vectors of ops 0, 1 and 4 (the
    # complex128 inverse) before any device call
    tree = (ctypes.c_int32 * 5)(0, 4, -1, -1, 0)
    rank = (ctypes.c_int32 * 1)(0)
    gens = (ctypes.c_double * 32)()
    for op in (-1, 6):
        assert L.hssx_hss_eval(0, _lib.HSSX_C64, 4, 1, tree, rank, gens, op, 1, ctypes.c_void_p(8),
                               ctypes.c_void_p(8), 0, None, None, None) == -1
    for op in (0, 1, 4):
        assert L.hssx_hss_eval(0, _lib.HSSX_C64, 4, 1, tree, rank, gens, op, 1, None, None, 0,
                               None, None, None) == -1
    assert L.hssx_hss_eval(0, _lib.HSSX_C64, 4, 1, tree, rank, gens, 5, 0, None, None, 3, None,
                           None, None) == -1
