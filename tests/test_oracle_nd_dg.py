"""Pins of the oracle's nested dissection on the discontinuous mesh (whole
triangles as units, Sec. 3.3 and Fig. 5 left): Definition 3.1 on the DG
matrix pattern, well-separated siblings, the element-conforming cluster
trees, and the rank-0 (block-diagonal) coupling of sibling separators."""
import numpy as np
import pytest

from oracle import fem_dg, nd


def _ancestors(tree, k):
    out = set()
    p = tree.boxes[k].parent
    while p >= 0:
        out.add(p)
        p = tree.boxes[p].parent
    return out


def test_c3_shapes():
    """SIPG-P2 on 256 x 256 x 2 triangles, leaves <= 10 triangles: 32,767
    nodes, depth 14, root separator 3,072 DOFs (two columns of 256 triangles
    facing the cut), widest boundary 1,914 DOFs."""
    t = nd.build_nd_dg(256, 60, 60)
    assert len(t.boxes) == 32767
    assert max(b.depth for b in t.boxes) == 14
    assert t.boxes[-1].I.size == 3072
    assert max(b.B.size for b in t.boxes) == 1914
    assert t.perm.size == 786432


@pytest.mark.parametrize("Nc,leaf", [(3, 12), (5, 24), (8, 60), (11, 36)])
def test_definition_3_1(Nc, leaf):
    t = nd.build_nd_dg(Nc, leaf, 12)
    A = fem_dg.assemble_dg(Nc, 1.0)
    n = A.shape[0]
    assert np.array_equal(np.sort(t.perm), np.arange(n))
    owner = np.empty(n, dtype=np.int64)
    for k, b in enumerate(t.boxes):
        owner[b.I] = k
    anc = [_ancestors(t, k) for k in range(len(t.boxes))]
    Ac = A.tocoo()
    for i, j in zip(Ac.row, Ac.col):
        a, c = owner[i], owner[j]
        if a != c:
            assert a in anc[c] or c in anc[a]
    for k, b in enumerate(t.boxes):
        assert set(owner[b.B].tolist()) <= anc[k]
        # an element's DOFs are never separated
        for v in (b.I, b.B):
            assert v.size % 6 == 0
            assert np.all(v.reshape(-1, 6) // 6 == (v.reshape(-1, 6) // 6)[:, :1])
        if not b.is_leaf:
            assert np.intersect1d(t.boxes[b.lo].B, t.boxes[b.hi].B).size == 0


def test_cluster_trees_conform_to_elements():
    t = nd.build_nd_dg(32, 60, 60)
    for b in t.boxes[:-1]:
        ct = b.ctree
        assert (ct.size % 6 == 0).all() and (ct.start % 6 == 0).all()
        assert (ct.size[ct.leaves()] <= 60).all()
        par = t.boxes[b.parent]
        assert set(b.B[:b.p0].tolist()) <= set(par.I.tolist())
        assert set(b.B[b.p0:].tolist()) <= set(par.B.tolist())


def test_dg_coupling_element_to_element():
    """Sibling separators couple element to element (each triangle of mu's
    interior part meets at most one triangle of nu's), and facing parts are
    clustered in step: cluster c of mu's interior tree meets nu's interior
    part outside cluster c through at most one element.  (A corner triangle
    that also faces the parent's boundary stays in B, which can shift the
    pairing by one element at the ends.)"""
    from oracle.hss import subtree
    Nc = 32
    t = nd.build_nd_dg(Nc, 60, 60)
    A = fem_dg.assemble_dg(Nc, 1.0).tocsr()
    checked = 0
    for b in t.boxes:
        if b.is_leaf or b.parent < 0:
            continue
        mu, nu = t.boxes[b.lo], t.boxes[b.hi]
        Pm, Pn = mu.B[:mu.p0], nu.B[:nu.p0]
        C = (A[Pm][:, Pn] != 0).astype(np.int64)
        E = np.add.reduceat(np.add.reduceat(C.toarray(), np.arange(0, Pm.size, 6), axis=0),
                            np.arange(0, Pn.size, 6), axis=1) if Pm.size and Pn.size else None
        if E is None:
            continue
        assert ((E > 0).sum(axis=1) <= 1).all() and ((E > 0).sum(axis=0) <= 1).all()
        cts = []
        for c in (mu, nu):
            ct = c.ctree
            cts.append(ct if c.p0 == c.B.size else subtree(ct, int(ct.left[0])))
        tm, tn = cts
        if tm.nclusters != tn.nclusters:
            continue
        for c in range(tm.nclusters):
            r0, r1 = tm.start[c] // 6, (tm.start[c] + tm.size[c]) // 6
            c0, c1 = tn.start[c] // 6, (tn.start[c] + tn.size[c]) // 6
            inside = E[r0:r1, c0:c1].astype(bool).sum()
            assert (E[r0:r1] > 0).sum() - inside <= 1
        checked += 1
    assert checked > 50
