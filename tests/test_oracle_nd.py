"""Pins of the oracle's nested dissection against Definition 3.1, the
well-separated property (Sec. 3.1) and the rank-1 coupling structure of
continuous Galerkin separators (Sec. 3.3)."""
import numpy as np
import pytest

from oracle import nd


def _ancestors(tree, k):
    out = set()
    p = tree.boxes[k].parent
    while p >= 0:
        out.add(p)
        p = tree.boxes[p].parent
    return out


def test_c1_c2_shapes():
    t = nd.build_nd(65, 32, 16)
    assert len(t.boxes) == 287
    assert max(b.depth for b in t.boxes) == 8
    assert sum(b.is_leaf for b in t.boxes) == 144
    assert t.boxes[-1].I.size == 130
    assert max(b.B.size for b in t.boxes) == 80


@pytest.mark.parametrize("N,leaf", [(9, 8), (17, 32), (33, 32), (40, 20)])
def test_definition_3_1(N, leaf):
    t = nd.build_nd(N, leaf, 8)
    n = N * N
    assert np.array_equal(np.sort(t.perm), np.arange(n))     # disjoint + cover
    owner = np.empty(n, dtype=np.int64)
    for k, b in enumerate(t.boxes):
        owner[b.I] = k
    indptr, idx = nd.grid_pattern(N)
    anc = [_ancestors(t, k) for k in range(len(t.boxes))]
    for i in range(n):
        for j in idx[indptr[i]:indptr[i + 1]]:
            a, c = owner[i], owner[j]
            if a != c:                        # coupled nodes: one is an ancestor
                assert a in anc[c] or c in anc[a]
    for k, b in enumerate(t.boxes):
        # B(sigma) is eliminated by ancestors and contains every ancestor DOF
        # coupled to I(sigma) (it may also hold box-corner DOFs with no such
        # coupling: B is the whole box boundary, see module docstring)
        assert set(owner[b.B].tolist()) <= anc[k]
        coupled = set()
        for i in b.I:
            for j in idx[indptr[i]:indptr[i + 1]]:
                if owner[j] in anc[k]:
                    coupled.add(int(j))
        assert coupled <= set(b.B.tolist())
        if not b.is_leaf:                     # well separated siblings
            assert np.intersect1d(t.boxes[b.lo].B, t.boxes[b.hi].B).size == 0


@pytest.mark.parametrize("N,beta", [(65, 16), (33, 8), (129, 16)])
def test_cluster_trees(N, beta):
    t = nd.build_nd(N, 32, beta)
    for b in t.boxes[:-1]:
        ct = b.ctree
        leaves = ct.leaves()
        assert (ct.size[leaves] <= beta).all()
        # leaves tile 0..|B|-1 in order; children split their parent's range
        assert np.array_equal(np.sort(ct.start[leaves]), np.cumsum(
            np.r_[0, ct.size[leaves][np.argsort(ct.start[leaves])]])[:-1])
        for c in range(ct.nclusters):
            if ct.left[c] >= 0:
                l, r = ct.left[c], ct.right[c]
                assert ct.start[l] == ct.start[c]
                assert ct.start[r] == ct.start[l] + ct.size[l]
                assert ct.size[l] + ct.size[r] == ct.size[c]
        # top split: P0 = B n I(parent) first
        par = t.boxes[b.parent]
        assert set(b.B[:b.p0].tolist()) <= set(par.I.tolist())
        assert set(b.B[b.p0:].tolist()) <= set(par.B.tolist())


def test_cg_coupling_rank_one():
    """Each cluster of mu's interior tree couples to nu's interior part only
    inside the cluster at the same tree position, up to one nonzero."""
    from oracle.hss import subtree
    N = 129
    t = nd.build_nd(N, 32, 16)
    indptr, idx = nd.grid_pattern(N)
    checked = 0
    for b in t.boxes:
        if b.is_leaf or b.parent < 0:
            continue
        mu, nu = t.boxes[b.lo], t.boxes[b.hi]
        cts = []
        for c in (mu, nu):
            ct = c.ctree
            cts.append(ct if c.p0 == c.B.size else subtree(ct, int(ct.left[0])))
        tm, tn = cts
        if tm.nclusters != tn.nclusters:
            continue
        assert np.array_equal(tm.size, tn.size)
        Pm, Pn = mu.B[:mu.p0], nu.B[:nu.p0]
        pos_n = {int(v): i for i, v in enumerate(Pn)}
        for c in range(tm.nclusters):
            rows = Pm[tm.start[c]:tm.start[c] + tm.size[c]]
            lo, hi = tn.start[c], tn.start[c] + tn.size[c]
            outside = 0
            for i in rows:
                for j in idx[indptr[i]:indptr[i + 1]]:
                    p = pos_n.get(int(j))
                    if p is not None and not (lo <= p < hi):
                        outside += 1
            assert outside <= 1
            checked += 1
    assert checked > 100
