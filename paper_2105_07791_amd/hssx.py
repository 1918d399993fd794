"""Python binding of the hssx C ABI: argument marshalling only.

Device buffers are torch CUDA tensors (complex128 vectors, float64 fields),
streams are torch streams; every computation runs in libhssx.so.
"""
import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import check, lib
from .symbolic import read_perm, read_tree

__all__ = ["Operator", "ElasticOperator", "DGOperator", "BatchOperator", "Factor", "assemble", "factor", "gmres_solve"]


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _col_major(x, dtype):
    """(n,) or (n, nrhs) tensor -> column-major (ptr, ld, nrhs, keepalive)."""
    if x.dim() == 1:
        x = x.reshape(-1, 1)
    t = x.t().resolve_conj()
    if not t.is_contiguous():
        t = t.contiguous()
    assert t.dtype == dtype and t.is_cuda
    return t, x.shape[0], x.shape[1]


class _OperatorBase:
    """Calls shared by single-problem and batch operators (handle, n, device)."""

    def __del__(self):
        if getattr(self, "handle", None) and getattr(_lib, "_LIB", None) is not None:
            lib().hssx_op_destroy(self.handle)
            self.handle = None

    def load(self, f, stream=None):
        """b = M f for nodal source samples f (n,) or (n, nrhs) float64."""
        f = torch.as_tensor(f, dtype=torch.float64, device=f"cuda:{self.device}")
        ft, n, nrhs = _col_major(f, torch.float64)
        b = torch.empty((nrhs, n), dtype=torch.complex128, device=f.device)
        check(lib().hssx_load(self.handle, nrhs, C.c_void_p(ft.data_ptr()), n,
                              C.c_void_p(b.data_ptr()), n, _stream(stream)))
        return b.t() if f.dim() == 2 else b[0]

    def matvec(self, x, stream=None):
        xt, n, nrhs = _col_major(x, torch.complex128)
        y = torch.empty((nrhs, n), dtype=torch.complex128, device=x.device)
        check(lib().hssx_matvec(self.handle, 0, nrhs, C.c_void_p(xt.data_ptr()), n,
                                C.c_void_p(y.data_ptr()), n, _stream(stream)))
        return y.t() if x.dim() == 2 else y[0]

    def csr(self):
        """(rowptr, col, val) as numpy arrays (host copies)."""
        nnz = C.c_long()
        check(lib().hssx_get_csr(self.handle, None, None, None, C.byref(nnz), None))
        rp = np.empty(self.n + 1, dtype=np.int32)
        col = np.empty(nnz.value, dtype=np.int32)
        val = np.empty(2 * nnz.value, dtype=np.float64)
        check(lib().hssx_get_csr(self.handle, rp.ctypes.data_as(_lib._ip),
                                 col.ctypes.data_as(_lib._ip), val.ctypes.data_as(_lib._dp),
                                 None, _stream()))
        return rp, col, val.view(np.complex128)

    def dAds_contract(self, lam, x, grad=None, adjoint=False, stream=None):
        """grad += -Re sum_rhs lam^T (dA/ds) x, or with adjoint=True
        -Re sum_rhs lam^H (dA/ds) x (lam the adjoint state A^-H dJ/dx)."""
        lt, n, nrhs = _col_major(lam, torch.complex128)
        xt, _, _ = _col_major(x, torch.complex128)
        if grad is None:
            grad = torch.zeros(n, dtype=torch.float64, device=lt.device)
        fn = lib().hssx_dAds_contract_adjoint if adjoint else lib().hssx_dAds_contract
        check(fn(self.handle, nrhs, C.c_void_p(lt.data_ptr()), C.c_void_p(xt.data_ptr()),
                 C.c_void_p(grad.data_ptr()), _stream(stream)))
        return grad


class Operator(_OperatorBase):
    """A(s) = K - omega^2 M[s^2] - i omega G[s] on the N x N P1 grid."""
    parts = 1

    def __init__(self, N, omega, slowness, device=0, stream=None):
        s = torch.as_tensor(slowness, dtype=torch.float64, device=f"cuda:{device}").contiguous()
        assert s.numel() == N * N
        self.N, self.omega, self.n, self.device = N, float(omega), N * N, device
        self.slowness = s
        self.part_off = [0, self.n]
        h = C.c_void_p()
        desc = _lib.ProblemDesc(N, float(omega))
        check(lib().hssx_assemble(device, C.byref(desc), C.c_void_p(s.data_ptr()),
                                  _stream(stream), C.byref(h)))
        self.handle = h


class ElasticOperator(_OperatorBase):
    """A = K[lam, mu] - omega^2 M[rho] - i omega C on the N x N P1 grid,
    2 unknowns per node (DOF 2 * node + component)."""
    parts = 1

    def __init__(self, N, omega, lam, mu, rho, device=0, stream=None):
        t = lambda a: torch.as_tensor(a, dtype=torch.float64,  # noqa: E731
                                      device=f"cuda:{device}").contiguous()
        lam, mu, rho = t(lam), t(mu), t(rho)
        assert lam.numel() == mu.numel() == rho.numel() == N * N
        self.N, self.omega, self.n, self.device = N, float(omega), 2 * N * N, device
        self.fields = (lam, mu, rho)
        self.part_off = [0, self.n]
        h = C.c_void_p()
        desc = _lib.ProblemDesc(N, float(omega))
        check(lib().hssx_assemble_elastic(device, C.byref(desc), C.c_void_p(lam.data_ptr()),
                                          C.c_void_p(mu.data_ptr()), C.c_void_p(rho.data_ptr()),
                                          _stream(stream), C.byref(h)))
        self.handle = h


class DGOperator(_OperatorBase):
    """SIPG Helmholtz operator on Nc x Nc x 2 triangles with P2 (default) or
    P1 elements (DOF nb e + a, nb = 6 or 3) and an absorbing (default) or
    homogeneous Dirichlet boundary; slowness given at the (Nc+1)^2 mesh
    vertices (None: 1)."""
    parts = 1

    def __init__(self, Nc, omega, slowness=None, p=2, bc="absorbing", device=0, stream=None):
        if slowness is None:
            slowness = torch.ones((Nc + 1) ** 2, dtype=torch.float64)
        s = torch.as_tensor(slowness, dtype=torch.float64, device=f"cuda:{device}").contiguous()
        assert s.numel() == (Nc + 1) ** 2
        nb = 3 if p == 1 else 6
        self.N, self.omega, self.n, self.device = Nc, float(omega), 2 * nb * Nc * Nc, device
        self.p, self.bc = p, bc
        self.slowness = s
        self.part_off = [0, self.n]
        h = C.c_void_p()
        code = {"absorbing": _lib.BC_ABSORBING, "dirichlet": _lib.BC_DIRICHLET}[bc]
        desc = _lib.IpdgDesc(Nc, p, code, float(omega))
        check(lib().hssx_assemble_ipdg(device, C.byref(desc), C.c_void_p(s.data_ptr()),
                                       _stream(stream), C.byref(h)))
        self.handle = h


class BatchOperator(_OperatorBase):
    """Independent problems as one block-diagonal operator (hssx_op_batch):
    vectors are the parts' vectors stacked, part p at rows part_off[p]:part_off[p+1]."""

    def __init__(self, operators, stream=None):
        ops = list(operators)
        arr = (C.c_void_p * len(ops))(*[o.handle for o in ops])
        h = C.c_void_p()
        check(lib().hssx_op_batch(len(ops), arr, _stream(stream), C.byref(h)))
        self.handle = h
        self.device = ops[0].device
        n, np_ = C.c_int(), C.c_int()
        check(lib().hssx_op_info(h, C.byref(n), C.byref(np_), None))
        off = np.empty(np_.value + 1, dtype=np.int32)
        check(lib().hssx_op_info(h, None, None, off.ctypes.data_as(_lib._ip)))
        self.n, self.parts, self.part_off = n.value, np_.value, [int(v) for v in off]
        self.Ns = [o.N for o in ops]
        self.omegas = [o.omega for o in ops]

    def split(self, x):
        """Views of the parts of a stacked vector (n,) or (n, nrhs)."""
        return [x[self.part_off[p]:self.part_off[p + 1]] for p in range(self.parts)]

class Factor:
    """Approximate factorization P = LDR of an Operator (Algorithm 3.4)."""

    def __init__(self, A, tol=1e-6, leaf_size=32, beta=16, h_sw=4, k0=32, r=16,
                 max_rounds=32, dtype="c128", seed=0, id_rel_tol=0.0, apply_graph=True,
                 autotune=True, sample_bf16=False, strict_tol=False, switch_size=0,
                 wide_inverse=False, stream=None):
        self.A = A
        opts = _lib.FactorOpts(beta, h_sw, k0, r, max_rounds,
                               _lib.HSSX_C128 if dtype == "c128" else _lib.HSSX_C64,
                               seed, id_rel_tol, int(apply_graph), int(autotune),
                               int(sample_bf16),  # 0, 1 (bf16) or 2 (split bf16)
                               int(switch_size), int(strict_tol), int(wide_inverse))
        h = C.c_void_p()
        check(lib().hssx_factor(A.handle, float(tol), int(leaf_size), C.byref(opts),
                                _stream(stream), C.byref(h)))
        self.handle = h

    def refactor(self, A=None, stream=None):
        """Numeric refactorization for A (default: the current operator),
        which must share the factor's pattern (hssx_refactor)."""
        A = self.A if A is None else A
        check(lib().hssx_refactor(self.handle, A.handle, _stream(stream)))
        self.A = A
        return self

    def __del__(self):
        if getattr(self, "handle", None) and getattr(_lib, "_LIB", None) is not None:
            lib().hssx_fact_destroy(self.handle)
            self.handle = None

    def apply(self, x, trans=False, stream=None):
        xt, n, nrhs = _col_major(x, torch.complex128)
        y = torch.empty((nrhs, n), dtype=torch.complex128, device=x.device)
        check(lib().hssx_apply(self.handle, int(trans), nrhs, C.c_void_p(xt.data_ptr()), n,
                               C.c_void_p(y.data_ptr()), n, _stream(stream)))
        return y.t() if x.dim() == 2 else y[0]

    def apply_noalloc(self, x, trans=False, stream=None):
        """apply() through hssx_apply_noalloc (no device allocation in the
        library; y is allocated here by torch)."""
        xt, n, nrhs = _col_major(x, torch.complex128)
        y = torch.empty((nrhs, n), dtype=torch.complex128, device=x.device)
        check(lib().hssx_apply_noalloc(self.handle, int(trans), nrhs, C.c_void_p(xt.data_ptr()),
                                       n, C.c_void_p(y.data_ptr()), n, _stream(stream)))
        return y.t() if x.dim() == 2 else y[0]

    def stats(self):
        s = _lib.FactorStats()
        check(lib().hssx_get_factor_stats(self.handle, C.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def perm(self):
        return read_perm(self.handle, self.A.n)

    def tree(self):
        """Flattened elimination and cluster trees (see hssx_get_tree)."""
        return read_tree(self.handle)

    def schur(self, node, nb):
        S = np.empty((nb, nb), dtype=np.complex128, order="F")
        check(lib().hssx_get_schur(self.handle, int(node),
                                   S.ctypes.data_as(_lib._dp), nb))
        return S


def gmres_solve(A, P, b, m=50, tol=1e-8, maxit=1000, flexible=False, trans=False, stream=None):
    """Preconditioned restarted GMRES; returns (x, list of per-system stats).
    A system is one right-hand side of one problem: entry r * A.parts + p.
    trans: False (A x = b), True (A^T x = b) or "adjoint" (A^H x = b)."""
    bt, n, nrhs = _col_major(b, torch.complex128)
    x = torch.empty((nrhs, n), dtype=torch.complex128, device=b.device)
    opts = _lib.GmresOpts(m, tol, maxit, int(flexible))
    stats = (_lib.GmresStats * (nrhs * A.parts))()
    tr = 2 if trans == "adjoint" else int(bool(trans))
    code = lib().hssx_gmres_solve(A.handle, P.handle if P is not None else None, tr, nrhs,
                                  C.c_void_p(bt.data_ptr()), n, C.c_void_p(x.data_ptr()), n,
                                  C.byref(opts), stats, _stream(stream))
    check(code)
    st = [dict(iters=s.iters, converged=bool(s.converged), prec_res=s.prec_res,
               true_res=s.true_res) for s in stats]
    return (x.t() if b.dim() == 2 else x[0]), st


def hss_eval(tree, rank, gens, op, X=None, ij=None, dtype="c128", device=0, stream=None):
    """hssx_hss_eval on one HSS matrix in generator form: tree int32 (ncl, 5)
    rows (start, size, left, right, level); rank int32 (ncl,); gens complex128
    packed as in include/hssx.h.  op 0: H X, 1: H^-1 X (X a complex128 device
    tensor (m,) or (m, nrhs)); op 2: H(i, j), 3: H^-1(i, j) for the rows of ij
    (int (n, 2)), returned as a complex128 numpy array; ops 4 and 5: ops 1 and 3
    with the inverse computed in complex128."""
    tree = np.ascontiguousarray(tree, dtype=np.int32)
    rank = np.ascontiguousarray(rank, dtype=np.int32)
    g = np.ascontiguousarray(np.asarray(gens, dtype=np.complex128)).view(np.float64)
    m, ncl = int(tree[0, 1]), int(tree.shape[0])
    dt = _lib.HSSX_C128 if dtype == "c128" else _lib.HSSX_C64
    args = (device, dt, m, ncl, tree.ctypes.data_as(_lib._ip), rank.ctypes.data_as(_lib._ip),
            g.ctypes.data_as(_lib._dp), int(op))
    if op in (0, 1, 4):
        xt, n, nrhs = _col_major(X, torch.complex128)
        y = torch.empty((nrhs, n), dtype=torch.complex128, device=X.device)
        check(lib().hssx_hss_eval(*args, nrhs, C.c_void_p(xt.data_ptr()), C.c_void_p(y.data_ptr()),
                                  0, None, None, _stream(stream)))
        return y.t() if X.dim() == 2 else y[0]
    ijc = np.ascontiguousarray(ij, dtype=np.int32)
    vals = np.empty(ijc.shape[0], dtype=np.complex128)
    check(lib().hssx_hss_eval(*args, 0, None, None, ijc.shape[0], ijc.ctypes.data_as(_lib._ip),
                              vals.view(np.float64).ctypes.data_as(_lib._dp), _stream(stream)))
    return vals


class Context:
    """A library context whose device memory comes from torch's caching
    allocator (hssx_create with an allocator that calls
    torch.cuda.caching_allocator_alloc / _delete).  Use as a context
    manager: handles created inside belong to it; destroy them before the
    context.  alloc_calls / free_calls / live count what passed through."""

    def __init__(self, device=0):
        self.device = device
        self.alloc_calls = self.free_calls = 0
        self.alloc_bytes = self.free_bytes = 0

        def _alloc(nbytes, stream, user):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                       int(stream or 0))
            except RuntimeError:
                return None
            self.alloc_calls += 1
            self.alloc_bytes += int(nbytes)
            return p

        def _free(ptr, nbytes, stream, user):
            torch.cuda.caching_allocator_delete(ptr)
            self.free_calls += 1
            self.free_bytes += int(nbytes)

        self._fns = (_lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free))   # kept alive
        self._spec = _lib.Allocator(self._fns[0], self._fns[1], None)
        h = C.c_void_p()
        check(lib().hssx_create(device, C.byref(self._spec), C.byref(h)))
        self.handle = h

    def __enter__(self):
        check(lib().hssx_bind(self.handle))
        return self

    def __exit__(self, *exc):
        check(lib().hssx_bind(None))
        return False

    def stats(self):
        live, a, f = C.c_long(), C.c_long(), C.c_long()
        check(lib().hssx_ctx_stats(self.handle, C.byref(live), C.byref(a), C.byref(f)))
        return {"live_bytes": live.value, "allocs": a.value, "frees": f.value}

    def destroy(self):
        if getattr(self, "handle", None):
            lib().hssx_destroy(self.handle)
            self.handle = None


def assemble(N, omega, slowness, device=0):
    return Operator(N, omega, slowness, device)


def factor(A, tol=1e-6, leaf_size=32, **kw):
    return Factor(A, tol, leaf_size, **kw)
