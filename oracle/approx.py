"""Approximate factorization P = LDR with HSS-compressed Schur complements
(oracle; Algorithm 3.4).

Per node sigma in post-order, with h_sw the switching height:

  * arithmetic class: HSS when height(sigma) > h_sw, dense otherwise;
  * a non-root node compresses its Schur complement when its parent uses HSS
    arithmetic ("form S densely and compress" below the switch, "form S
    directly in HSS form" above it);
  * dense class: the front is assembled from the children's (dense or
    expanded) Schur complements and A, A_ii is LU-factored, R = -A_ii^-1 A_ib,
    L = R^T, S = A_bb + A_bi R (eqs. 3.2-3.5);
  * HSS class (Sec. 3.3, Algorithm 3.3): with A_ii = [[S_ii^mu, A~^(mu,nu)],
    [A~^(nu,mu), S_ii^nu]], the inner Schur complement
    S~ = S_ii^nu - A~^(nu,mu) (S_ii^mu)^-1 A~^(mu,nu) is compressed with
    Algorithm A.1 on nu's interior cluster tree, and A_ii^-1 is applied by
    the 2x2 block elimination of Algorithm 3.2 with S~ replaced by its HSS
    approximation.  R = -A_ii^-1 A_ib, L = R^T (Sec. 3.4), and
    S = A_bb + A_bi R is compressed with Algorithm A.1 (Sec. 3.5);
  * the root (either class) factors its dense A_ii (Sec. 3.1, last remark of
    the elimination), expanding HSS children when needed.

The oracle forms every operator densely and inverts the HSS-represented
blocks exactly (plain definition of the HSS arithmetic), so it carries the
same approximations as the compressed method: the two Algorithm A.1 calls
per HSS node and the one per transition node, with the same random sketches
(instance keys 4*node+0 for S, 4*node+1 for S~).

Symmetry: A is complex symmetric, every compressed operator is symmetric,
so L = R^T and the transpose apply reuses the same blocks.
"""
import numpy as np
import scipy.linalg as sla

from .hss import compress_adaptive, subtree

__all__ = ["ApproxFactor", "factor_approx", "apply_ldr"]


def apply_ldr(tree, solve_ii, L, R, b, trans=False):
    """Algorithm 3.1: bottom-up L sweep, block-diagonal solve, top-down R
    sweep (or the transposed sequence).  b in natural node numbering."""
    x = np.array(b, dtype=np.complex128, copy=True)
    vec = x.ndim == 1
    if vec:
        x = x[:, None]
    boxes = tree.boxes
    first, last = (R, L) if trans else (L, R)
    for k, bx in enumerate(boxes):
        if bx.B.size and bx.I.size:
            blk = first[k].T if trans else first[k]
            x[bx.B] += blk @ x[bx.I]
    for k, bx in enumerate(boxes):
        if bx.I.size:
            x[bx.I] = solve_ii(k, x[bx.I], trans)
    for k in range(len(boxes) - 1, -1, -1):
        bx = boxes[k]
        if bx.B.size and bx.I.size:
            blk = last[k].T if trans else last[k]
            x[bx.I] += blk @ x[bx.B]
    return x[:, 0] if vec else x


class _Block2x2:
    """A_ii^-1 by Algorithm 3.2 with dense inverses of B11 and of the
    HSS-approximated inner Schur complement."""

    def __init__(self, B11, B12, B21, S_tilde_hss_dense):
        self.p = B11.shape[0]
        self.lu11 = sla.lu_factor(B11)
        self.B12 = B12
        self.B21 = B21
        self.luS = sla.lu_factor(S_tilde_hss_dense)

    def solve(self, X, trans=False):
        """Algorithm 3.2; the approximated A_ii is symmetric, so the
        transposed solve is the same map."""
        p = self.p
        X1 = sla.lu_solve(self.lu11, X[:p])
        X2 = X[p:] - self.B21 @ X1
        X2 = sla.lu_solve(self.luS, X2)
        X1 = X1 - sla.lu_solve(self.lu11, self.B12 @ X2)
        return np.vstack([X1, X2])


class ApproxFactor:
    def __init__(self, tree, h_sw):
        self.tree = tree
        self.h_sw = h_sw
        self.arith, self.comp = tree.classes(h_sw)
        self.lu = {}
        self.blk = {}
        self.L = {}
        self.R = {}
        self.S_dense = {}
        self.S_hss = {}
        self.S_tilde = {}
        self.stats = {}

    def solve_ii(self, k, X, trans=False):
        if k in self.blk:
            return self.blk[k].solve(X, trans)
        return sla.lu_solve(self.lu[k], X, trans=1 if trans else 0)

    def apply(self, b):
        return apply_ldr(self.tree, self.solve_ii, self.L, self.R, b)

    def apply_t(self, b):
        return apply_ldr(self.tree, self.solve_ii, self.L, self.R, b, trans=True)

    def child_S(self, c):
        if c in self.S_hss:
            return self.S_hss[c].dense()
        return self.S_dense[c]

    def k_max(self):
        ks = [h.max_rank() for h in self.S_hss.values()]
        ks += [h.max_rank() for h in self.S_tilde.values()]
        return max(ks, default=0)


def _front(A, tree, k, child_S):
    bx = tree.boxes[k]
    front = np.concatenate([bx.I, bx.B])
    F = A[front][:, front].toarray().astype(np.complex128)
    if not bx.is_leaf:
        pos = np.full(tree.perm.size, -1, dtype=np.int64)
        pos[front] = np.arange(front.size)
        for c in (bx.lo, bx.hi):
            p = pos[tree.boxes[c].B]
            F[np.ix_(p, p)] = child_S(c)
    return F


def _interior_tree(box):
    """Cluster tree of the P0 part of a node's boundary (its S_ii block)."""
    ct = box.ctree
    if ct.nclusters == 0 or box.p0 == 0:     # no P0 part: empty tree
        return type(ct)(*(np.zeros(0, np.int64) for _ in range(5)))
    if box.p0 == box.B.size:                 # no P1 part: the whole tree
        return ct
    return subtree(ct, int(ct.left[0]))


def factor_approx(A, tree, h_sw=4, tol=1e-6, k0=32, r=16, seed=0,
                  id_rel_tol=None):
    """Algorithm 3.4.  Every Algorithm A.1 call starts from the rank guess
    max(k0, accepted k of the children's Schur-complement compressions): the
    rank of a parent's Schur complement grows slowly up the tree."""
    f = ApproxFactor(tree, h_sw)
    root = tree.root
    kfin = {}
    for k, bx in enumerate(tree.boxes):
        F = _front(A, tree, k, f.child_S)
        ni = bx.I.size
        Aii, Aib = F[:ni, :ni], F[:ni, ni:]
        Abi, Abb = F[ni:, :ni], F[ni:, ni:]
        if f.arith[k] == "hss" and k != root and ni > tree.boxes[bx.lo].p0:
            mu = tree.boxes[bx.lo]
            p = mu.p0
            B11, B12 = Aii[:p, :p], Aii[:p, p:]
            B21, B22 = Aii[p:, :p], Aii[p:, p:]
            lu11 = sla.lu_factor(B11)
            St = B22 - B21 @ sla.lu_solve(lu11, B12)
            ct = _interior_tree(tree.boxes[bx.hi])
            Ht = compress_adaptive(lambda X: St @ X,
                                   lambda I, J: St[np.ix_(I, J)], ct,
                                   k0=max(k0, kfin.get(bx.hi, 0)), r=r, tol=tol, seed=seed,
                                   instance=4 * k + 1, id_rel_tol=id_rel_tol)
            f.S_tilde[k] = Ht
            f.blk[k] = _Block2x2(B11, B12, B21, Ht.dense())
        elif ni:
            f.lu[k] = sla.lu_factor(Aii)
        if bx.B.size:
            if ni:
                R = -f.solve_ii(k, Aib)
                f.R[k] = R
                f.L[k] = R.T.copy()
                S = Abb + Abi @ R
            else:
                S = Abb.copy()
            if f.comp[k]:
                kc = 0 if bx.is_leaf else max(kfin.get(bx.lo, 0), kfin.get(bx.hi, 0))
                H = compress_adaptive(lambda X: S @ X,
                                      lambda I, J: S[np.ix_(I, J)], bx.ctree,
                                      k0=max(k0, kc), r=r, tol=tol, seed=seed,
                                      instance=4 * k, id_rel_tol=id_rel_tol)
                f.S_hss[k] = H
                kfin[k] = H.k_final
            else:
                f.S_dense[k] = S
        if not bx.is_leaf:
            for c in (bx.lo, bx.hi):
                f.S_dense.pop(c, None)
    return f
