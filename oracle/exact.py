"""Exact nested-dissection LDR elimination and its inverse (oracle).

This is the sparse direct solver the approximate method starts from
(Sec. 3.1, eqs. 3.2-3.5, Algorithm 3.1); with no compression the approximate
factorization reduces to it (Sec. 3.2 opening remark).

For every tree node sigma, in post-order:
  * the front A^(sigma) over [I(sigma); B(sigma)] is
      - a leaf: the entries A(front, front)                            (eq. 3.2)
      - a non-leaf with children mu, nu: S^(mu) on B(mu) x B(mu), S^(nu) on
        B(nu) x B(nu), and original entries A(p, q) across the two (eq. 3.4);
  * L = -A_bi A_ii^-1, R = -A_ii^-1 A_ib                              (eq. 3.3)
  * S = A_bb + A_bi R  (= A_bb - A_bi A_ii^-1 A_ib)                   (eq. 3.5)
  * the root keeps only A_ii.
Dense solves use LAPACK's LU with partial pivoting (scipy.linalg.lu_factor).
"""
import numpy as np
import scipy.linalg as sla

__all__ = ["ExactFactor", "factor_exact", "front_matrix"]


class ExactFactor:
    def __init__(self, tree):
        self.tree = tree
        self.lu = {}       # node -> lu_factor(A_ii)
        self.L = {}        # node -> L (|B| x |I|)
        self.R = {}        # node -> R (|I| x |B|)
        self.S = {}        # node -> S (|B| x |B|) (kept for tests)

    # Algorithm 3.1: b -> R^-1 D^-1 L^-1 b  (natural node numbering)
    def apply(self, b):
        x = np.array(b, dtype=np.complex128, copy=True)
        vec = x.ndim == 1
        if vec:
            x = x[:, None]
        boxes = self.tree.boxes
        for k, bx in enumerate(boxes):                       # bottom-up
            if bx.B.size and bx.I.size:
                x[bx.B] += self.L[k] @ x[bx.I]
        for k, bx in enumerate(boxes):                       # block diagonal
            if bx.I.size:
                x[bx.I] = sla.lu_solve(self.lu[k], x[bx.I])
        for k in range(len(boxes) - 1, -1, -1):              # top-down
            bx = boxes[k]
            if bx.B.size and bx.I.size:
                x[bx.I] += self.R[k] @ x[bx.B]
        return x[:, 0] if vec else x

    # transpose of Algorithm 3.1: b -> L^-T D^-T R^-T b
    def apply_t(self, b):
        x = np.array(b, dtype=np.complex128, copy=True)
        vec = x.ndim == 1
        if vec:
            x = x[:, None]
        boxes = self.tree.boxes
        for k, bx in enumerate(boxes):
            if bx.B.size and bx.I.size:
                x[bx.B] += self.R[k].T @ x[bx.I]
        for k, bx in enumerate(boxes):
            if bx.I.size:
                x[bx.I] = sla.lu_solve(self.lu[k], x[bx.I], trans=1)
        for k in range(len(boxes) - 1, -1, -1):
            bx = boxes[k]
            if bx.B.size and bx.I.size:
                x[bx.I] += self.L[k].T @ x[bx.B]
        return x[:, 0] if vec else x


def front_matrix(A, tree, k, S):
    """Dense front of node k over [I; B] (eqs. 3.2 / 3.4)."""
    bx = tree.boxes[k]
    front = np.concatenate([bx.I, bx.B])
    F = A[front][:, front].toarray().astype(np.complex128)
    if not bx.is_leaf:
        for c in (bx.lo, bx.hi):
            cb = tree.boxes[c].B
            pos = np.full(tree.perm.size, -1, dtype=np.int64)
            pos[front] = np.arange(front.size)
            p = pos[cb]
            assert (p >= 0).all()
            F[np.ix_(p, p)] = S[c]
    return F


def factor_exact(A, tree, keep_S=True):
    """Exact multifrontal factorization of the CSR matrix A (natural order)."""
    f = ExactFactor(tree)
    S = {}
    for k, bx in enumerate(tree.boxes):
        F = front_matrix(A, tree, k, S)
        ni = bx.I.size
        Aii, Aib = F[:ni, :ni], F[:ni, ni:]
        Abi, Abb = F[ni:, :ni], F[ni:, ni:]
        if ni:
            f.lu[k] = sla.lu_factor(Aii)
        if bx.B.size:
            if ni:
                f.R[k] = -sla.lu_solve(f.lu[k], Aib)
                f.L[k] = -sla.lu_solve(f.lu[k], Abi.T, trans=1).T
                S[k] = Abb + Abi @ f.R[k]
            else:
                S[k] = Abb.copy()
        if not bx.is_leaf:                      # children's S are consumed
            if not keep_S:
                S.pop(bx.lo, None)
                S.pop(bx.hi, None)
    if keep_S:
        f.S = S
    return f
