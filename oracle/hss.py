"""HSS matrices with interpolative bases, and their adaptive randomized
compression (oracle).

Representation (Sec. 2.2, eqs. 2.2-2.6) for a complex symmetric matrix
(A^T = A), so the column generators equal the row generators (V = U) and
transposes replace conjugate transposes (the paper states Algorithm A.1 for a
real symmetric matrix):

  * leaf cluster c:      D_c = A(I_c, I_c)
  * non-root cluster c:  U_c (rows_c x k_c) with U_c(J_c, :) = identity;
                         rows_c = |I_c| at a leaf, k_left + k_right otherwise;
                         skeleton sk_c = the k_c indices of I_c it keeps
  * internal cluster p with children l, r:
                         B12_p = A(sk_l, sk_r),  B21_p = A(sk_r, sk_l)
  so that A(I_l, I_r) = Ut_l B12_p Ut_r^T with the nested bases
  Ut_c = diag(Ut_left, Ut_right) U_c (eq. 2.3).

Compression (Sec. 2.3, Appendix A, Algorithm A.1): sample S = A Omega with
k + r Gaussian columns, walk the cluster tree bottom-up, remove the diagonal
(leaf) or sibling (internal) contribution from the local samples, take an
interpolative decomposition of the local sample rows, reduce Omega and the
samples to the skeleton, and read D and B from entries of A.  Then estimate
the error with r fresh probes (eq. 2.7); on failure set k <- k + r, append
the probes to Omega and S, and compress again.

Readings taken where the paper is silent or garbled:
  * the inner sibling block uses the children's skeleton sets at both
    indices (the printed superscripts disagree between two lines);
  * the loop also visits the root to read its B block; the root has no ID;
  * the ID is S_loc ~ U S_loc(J, :) with U(J, :) = I, computed by column-
    pivoted Householder QR of S_loc^T (pivot = largest remaining column norm,
    lowest original row index on ties); rank = min(k, rows, cols) and, additionally, the
    pivots whose magnitude falls below id_rel_tol * |first pivot| are dropped;
  * the tolerance is relative: accept when
    ||S~ - A_HSS Omega~||_F <= tol * ||S~||_F, S~ = A Omega~ the probe samples;
  * Omega has real N(0,1) entries (the estimator stays unbiased).
"""
import numpy as np
import scipy.linalg as sla

from .nd import ClusterTree
from .rng import gaussian_block

__all__ = ["HSS", "interp_decomp", "compress_adaptive", "compress_plain",
           "subtree", "random_hss"]


def subtree(ct, root_id):
    """The cluster tree rooted at cluster root_id, renumbered in level order
    with positions relative to its first index."""
    queue = [(root_id, 0)]
    k = 0
    while k < len(queue):
        c, lev = queue[k]
        k += 1
        if ct.left[c] >= 0:
            queue.append((ct.left[c], lev + 1))
            queue.append((ct.right[c], lev + 1))
    num = {c: i for i, (c, _) in enumerate(queue)}
    base = ct.start[root_id]
    a = lambda v: np.asarray(v, dtype=np.int64)
    return ClusterTree(
        a([ct.start[c] - base for c, _ in queue]),
        a([ct.size[c] for c, _ in queue]),
        a([num[ct.left[c]] if ct.left[c] >= 0 else -1 for c, _ in queue]),
        a([num[ct.right[c]] if ct.right[c] >= 0 else -1 for c, _ in queue]),
        a([lev for _, lev in queue]))


class HSS:
    def __init__(self, tree):
        self.tree = tree
        self.m = int(tree.size[0]) if tree.nclusters else 0
        self.D = {}
        self.U = {}
        self.sk = {}
        self.B12 = {}
        self.B21 = {}
        self.k_final = 0
        self.rounds = 0
        self.est = np.inf

    def ranks(self):
        return {c: self.U[c].shape[1] for c in self.U}

    def max_rank(self):
        return max((u.shape[1] for u in self.U.values()), default=0)

    def _children(self, c):
        return self.tree.left[c], self.tree.right[c]

    def _is_leaf(self, c):
        return self.tree.left[c] < 0

    def _range(self, c):
        s = self.tree.start[c]
        return np.arange(s, s + self.tree.size[c])

    def matvec(self, X):
        """Y = A X by the telescoping recursion (eqs. 2.5-2.6): up-sweep of
        the bases, sibling couplings, down-sweep, plus the leaf blocks."""
        X = np.asarray(X)
        vec = X.ndim == 1
        if vec:
            X = X[:, None]
        t = self.tree
        Y = np.zeros((self.m, X.shape[1]), dtype=np.result_type(X, np.complex128))
        if t.nclusters == 0:
            return Y[:, 0] if vec else Y
        order = np.argsort(-t.level, kind="stable")       # deepest first
        xh = {}
        for c in order:
            if c == 0:
                continue
            if self._is_leaf(c):
                xh[c] = self.U[c].T @ X[self._range(c)]
            else:
                l, r = self._children(c)
                xh[c] = self.U[c].T @ np.vstack([xh[l], xh[r]])
        yh = {c: 0 for c in range(t.nclusters)}
        for p in range(t.nclusters):
            if not self._is_leaf(p):
                l, r = self._children(p)
                yh[l] = yh[l] + self.B12[p] @ xh[r]
                yh[r] = yh[r] + self.B21[p] @ xh[l]
        for c in order[::-1]:                              # top-down
            if self._is_leaf(c):
                rg = self._range(c)
                Y[rg] = self.D[c] @ X[rg]
                if c != 0:
                    Y[rg] += self.U[c] @ yh[c]
            elif c != 0:
                l, r = self._children(c)
                z = self.U[c] @ yh[c]
                kl = self.U[l].shape[1]
                yh[l] = yh[l] + z[:kl]
                yh[r] = yh[r] + z[kl:]
        return Y[:, 0] if vec else Y

    def dense(self):
        """Dense expansion from the nested bases (eqs. 2.2-2.3), filling each
        sibling block Ut_l B12 Ut_r^T and each leaf block D."""
        t = self.tree
        A = np.zeros((self.m, self.m), dtype=np.complex128)
        if t.nclusters == 0:
            return A
        Ut = {}
        for c in np.argsort(-t.level, kind="stable"):
            if c == 0:
                continue
            if self._is_leaf(c):
                Ut[c] = self.U[c]
            else:
                l, r = self._children(c)
                Ut[c] = sla.block_diag(Ut[l], Ut[r]) @ self.U[c]
        for c in range(t.nclusters):
            if self._is_leaf(c):
                rg = self._range(c)
                A[np.ix_(rg, rg)] = self.D[c]
            else:
                l, r = self._children(c)
                rl, rr = self._range(l), self._range(r)
                A[np.ix_(rl, rr)] = Ut[l] @ self.B12[c] @ Ut[r].T
                A[np.ix_(rr, rl)] = Ut[r] @ self.B21[c] @ Ut[l].T
        return A


def interp_decomp(S, k, id_rel_tol=0.0):
    """Row interpolative decomposition S ~ U S[J, :], U[J, :] = I (eq. A.1 on
    the transpose).  Column-pivoted Householder QR of S^T; returns (U, J)."""
    S = np.asarray(S, dtype=np.complex128)
    m, s = S.shape
    M = S.T.copy()                         # columns of M are the rows of S
    perm = np.arange(m)
    kmax = min(k, m, s)
    first = None
    rank = 0
    for t in range(kmax):
        norms = np.sum(np.abs(M[t:, t:]) ** 2, axis=0)
        ties = np.flatnonzero(norms == norms.max())
        p = t + int(ties[np.argmin(perm[t + ties])])     # lowest original row on ties
        pn = np.sqrt(norms[p - t])
        if first is None:
            first = pn
        if pn == 0.0 or pn <= id_rel_tol * first:
            break
        if p != t:
            M[:, [t, p]] = M[:, [p, t]]
            perm[[t, p]] = perm[[p, t]]
        x = M[t:, t].copy()
        nx = np.linalg.norm(x)
        phase = x[0] / abs(x[0]) if x[0] != 0 else 1.0
        v = x.copy()
        v[0] += phase * nx
        vv = np.vdot(v, v).real
        if vv > 0:
            M[t:, t:] -= np.outer(v, (2.0 / vv) * (v.conj() @ M[t:, t:]))
        rank = t + 1
    R11 = np.triu(M[:rank, :rank])
    R12 = M[:rank, rank:]
    T = sla.solve_triangular(R11, R12) if rank else np.zeros((0, m))
    U = np.zeros((m, rank), dtype=np.complex128)
    U[perm[:rank], np.arange(rank)] = 1.0
    U[perm[rank:], :] = T.T
    return U, perm[:rank].copy()


def _compress_once(S, Omega, entries, tree, k, id_rel_tol):
    H = HSS(tree)
    Om, Sr = {}, {}
    for c in np.argsort(-tree.level, kind="stable"):     # bottom-up
        if H._is_leaf(c):
            I_loc = H._range(c)
            D = entries(I_loc, I_loc)
            H.D[c] = D
            Om_loc = Omega[I_loc]
            S_loc = S[I_loc] - D @ Om_loc
        else:
            l, r = H._children(c)
            I_loc = np.concatenate([H.sk[l], H.sk[r]])
            H.B12[c] = entries(H.sk[l], H.sk[r])
            H.B21[c] = entries(H.sk[r], H.sk[l])
            Om_loc = np.vstack([Om[l], Om[r]])
            S_loc = np.vstack([Sr[l] - H.B12[c] @ Om[r], Sr[r] - H.B21[c] @ Om[l]])
        if c == 0:
            break
        U, J = interp_decomp(S_loc, k, id_rel_tol)
        H.U[c] = U
        H.sk[c] = I_loc[J]
        Om[c] = U.T @ Om_loc
        Sr[c] = S_loc[J]
    return H


def compress_adaptive(apply, entries, tree, k0=32, r=16, tol=1e-6, seed=0,
                      instance=0, id_rel_tol=None, max_rounds=64):
    """Algorithm A.1.  apply(X) = A X for a real (m x c) X; entries(I, J) =
    A(I, J).  Returns the HSS approximation; .k_final, .rounds and .est hold
    the final rank parameter, number of compressions and relative estimate."""
    if id_rel_tol is None:
        id_rel_tol = 1e-2 * tol
    m = int(tree.size[0]) if tree.nclusters else 0
    k = max(1, min(k0, m))
    Omega = gaussian_block(seed, instance, m, 0, k + r)
    S = apply(Omega)
    col = k + r
    rounds = 0
    while True:
        H = _compress_once(S, Omega, entries, tree, k, id_rel_tol)
        rounds += 1
        Om_t = gaussian_block(seed, instance, m, col, r)
        col += r
        S_t = apply(Om_t)
        ref = np.linalg.norm(S_t)
        err = np.linalg.norm(S_t - H.matvec(Om_t))
        est = err / ref if ref > 0 else 0.0
        if est <= tol or k >= m or rounds >= max_rounds:
            H.k_final, H.rounds, H.est = k, rounds, est
            return H
        k += r
        Omega = np.hstack([Omega, Om_t])
        S = np.hstack([S, S_t])


def compress_plain(A, tree, tol):
    """Deterministic checker: IDs of the full HSS block rows A(I_loc, rest)
    bottom-up (the quadratic-cost construction), relative truncation tol."""
    A = np.asarray(A, dtype=np.complex128)
    m = A.shape[0]
    H = HSS(tree)
    for c in np.argsort(-tree.level, kind="stable"):
        rg = H._range(c)
        rest = np.setdiff1d(np.arange(m), rg)
        if H._is_leaf(c):
            I_loc = rg
            H.D[c] = A[np.ix_(rg, rg)]
        else:
            l, r = H._children(c)
            I_loc = np.concatenate([H.sk[l], H.sk[r]])
            H.B12[c] = A[np.ix_(H.sk[l], H.sk[r])]
            H.B21[c] = A[np.ix_(H.sk[r], H.sk[l])]
        if c == 0:
            break
        S_loc = A[np.ix_(I_loc, rest)]
        U, J = interp_decomp(S_loc, S_loc.shape[0], tol)
        H.U[c] = U
        H.sk[c] = I_loc[J]
    return H


def random_hss(tree, k, seed=0):
    """A random complex symmetric HSS matrix of rank <= k on the given tree
    (test input): random D (symmetrised), random interpolative U, random B."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H = HSS(tree)
    cplx = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    for c in np.argsort(-tree.level, kind="stable"):
        if H._is_leaf(c):
            rg = H._range(c)
            d = cplx(rg.size, rg.size)
            H.D[c] = d + d.T
            idx = rg
        else:
            l, r = H._children(c)
            idx = np.concatenate([H.sk[l], H.sk[r]])
            b = cplx(H.sk[l].size, H.sk[r].size)
            H.B12[c] = b
            H.B21[c] = b.T.copy()
        if c == 0:
            break
        kk = min(k, idx.size)
        J = np.sort(rng.choice(idx.size, size=kk, replace=False))
        U = cplx(idx.size, kk) * 0.5
        U[J] = np.eye(kk)
        H.U[c] = U
        H.sk[c] = idx[J]
    return H
