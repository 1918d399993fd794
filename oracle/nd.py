"""Box nested dissection, elimination tree and Schur-complement cluster trees
(oracle).  Integer work only; the HIP library implements the same rules
independently and the tests compare the two bit for bit.

Rules (Sec. 3.1 Def. 3.1 and Fig. 3; Sec. 3.2 Fig. 4; Sec. 3.3):

* Boxes are half-open node ranges [x0,x1) x [y0,y1); the root is the whole
  N x N grid.  A box with nx*ny*dofs_per_node <= leaf_dofs is a leaf.  Any
  other box is split across its longer side (tie -> split in x) at
  x0 + floor(nx/2) (resp. y), giving children (low, high).  Alternating the
  cut with the aspect ratio keeps boxes near square (Sec. 4.1).
* Tree nodes are numbered in post-order: low subtree, high subtree, self.
* Two grid nodes are adjacent when the matrix pattern couples them (they share
  a triangle).  Bd(sigma) = nodes of box sigma adjacent to a node outside it.
* Leaf: I = box minus Bd(sigma).  Non-leaf with children mu, nu:
  I = (Bd(mu) u Bd(nu)) minus Bd(sigma).  B = Bd(sigma); the root has B empty.
  Because boxes partition the grid, sibling boundaries are disjoint, which is
  the well-separated property the method relies on (Sec. 3.1, Fig. 3; elements
  straddling a cut are split between the boxes as for continuous Galerkin).
* Order of B(sigma) = leaf order of its cluster tree.  The top split puts
  P0 = B(sigma) n I(parent) first and P1 = B(sigma) n B(parent) second, so the
  block S_ii that the parent eliminates is a subtree (Fig. 4).  Each part is
  bisected until a cluster holds <= beta DOFs: axis x if
  (xmax-xmin) >= (ymax-ymin) else y, stable sort of the nodes by
  (axis coordinate, other coordinate, node id), split at floor(count/2).
  Facing parts of the two children are therefore clustered in step, which is
  what gives the coupling block its rank-1 HSS structure (Sec. 3.3).
* Order of I(sigma): a leaf sorts its nodes by (y, x); a non-leaf lists mu's P0
  then nu's P0 (the block layout of eq. 3.4).
* The elimination permutation concatenates I(sigma) over the post-order.
* With several unknowns per node (vector problems) every node contributes its
  components consecutively (DOF id = dofs * node + component); boxes and
  clusters are formed on nodes with sizes counted in DOFs.
* Discontinuous Galerkin (build_nd_dg): the same rules with boxes over mesh
  cells and whole triangles as the units (Sec. 3.3, Fig. 5 left), adjacency
  across faces, and the triangle centroids as cluster coordinates.
"""
from dataclasses import dataclass, field

import numpy as np

__all__ = ["Box", "ClusterTree", "NDTree", "build_nd", "build_nd_dg", "grid_pattern", "dg_pattern"]


def grid_pattern(N):
    """CSR structure (indptr, indices) of the P1 stencil on the N x N grid:
    node pairs sharing a triangle, including the diagonal."""
    from .fem import triangles
    n = N * N
    t = triangles(N)
    r = np.repeat(t, 3, axis=1).ravel()
    c = np.tile(t, 3).ravel()
    key = np.unique(r * n + c)
    rows = key // n
    cols = key % n
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    return np.cumsum(indptr), cols


@dataclass
class ClusterTree:
    """Binary cluster tree over positions 0..m-1 of an ordered index list,
    stored in level order.  start/size give each cluster's contiguous range;
    left/right are child cluster ids (-1 at leaves)."""
    start: np.ndarray
    size: np.ndarray
    left: np.ndarray
    right: np.ndarray
    level: np.ndarray

    @property
    def nclusters(self):
        return self.start.size

    def leaves(self):
        return np.nonzero(self.left < 0)[0]

    def depth(self):
        return int(self.level.max()) if self.level.size else 0


@dataclass
class Box:
    x0: int
    x1: int
    y0: int
    y1: int
    lo: int = -1
    hi: int = -1
    parent: int = -1
    depth: int = 0
    height: int = 0
    bd: np.ndarray = None          # sorted node ids of Bd(sigma)
    I: np.ndarray = None           # ordered interior node ids
    B: np.ndarray = None           # ordered boundary node ids (cluster order)
    p0: int = 0                    # |P0|: first p0 entries of B face the parent's I
    ctree: ClusterTree = None      # cluster tree over B
    offset: int = 0                # start of I in the permutation

    @property
    def is_leaf(self):
        return self.lo < 0


class _CNode:
    __slots__ = ("ids", "left", "right")

    def __init__(self, ids=None, left=None, right=None):
        self.ids, self.left, self.right = ids, left, right


def _bisect(units, coords, beta, dofs):
    """Recursive geometric bisection of a unit-id array into clusters;
    coords(ids) gives integer (x, y) per unit."""
    if units.size * dofs <= beta:
        return _CNode(ids=units)
    x, y = coords(units)
    if (x.max() - x.min()) >= (y.max() - y.min()):
        order = np.lexsort((units, y, x))     # primary x, then y, then id
    else:
        order = np.lexsort((units, x, y))     # primary y, then x, then id
    s = units[order]
    h = s.size // 2
    return _CNode(left=_bisect(s[:h], coords, beta, dofs),
                  right=_bisect(s[h:], coords, beta, dofs))


def _cluster_tree(parts, coords, beta, dofs):
    """Cluster tree (level order) and the leaf order of the listed parts.

    parts: list of unit-id arrays (P0, P1); empty parts are dropped.  With two
    non-empty parts the root splits them; otherwise the root is the single
    part's bisection."""
    subs = [_bisect(p, coords, beta, dofs) for p in parts if p.size > 0]
    empty = np.zeros(0, dtype=np.int64)
    if not subs:
        return ClusterTree(empty, empty, empty, empty, empty), empty
    root = subs[0] if len(subs) == 1 else _CNode(left=subs[0], right=subs[1])

    order = []
    rng = {}

    def walk(t):
        st = len(order)
        if t.left is None:
            order.extend(t.ids.tolist())
        else:
            walk(t.left)
            walk(t.right)
        rng[id(t)] = (st, len(order))

    walk(root)
    queue = [(root, 0)]
    k = 0
    while k < len(queue):                      # breadth-first numbering
        t, lev = queue[k]
        k += 1
        if t.left is not None:
            queue.append((t.left, lev + 1))
            queue.append((t.right, lev + 1))
    num = {id(t): i for i, (t, _) in enumerate(queue)}
    start = [rng[id(t)][0] for t, _ in queue]
    size = [rng[id(t)][1] - rng[id(t)][0] for t, _ in queue]
    left = [num[id(t.left)] if t.left is not None else -1 for t, _ in queue]
    right = [num[id(t.right)] if t.right is not None else -1 for t, _ in queue]
    level = [lev for _, lev in queue]
    a = lambda v: np.asarray(v, dtype=np.int64)
    return ClusterTree(a(start), a(size), a(left), a(right), a(level)), \
        np.asarray(order, dtype=np.int64)


@dataclass
class NDTree:
    N: int
    leaf_dofs: int
    beta: int
    dofs: int
    boxes: list = field(default_factory=list)   # post-order
    perm: np.ndarray = None                      # perm[k] = node id at position k
    iperm: np.ndarray = None

    @property
    def root(self):
        return len(self.boxes) - 1

    def classes(self, h_sw):
        """Per node: arith in {'dense','hss'} and whether S is compressed.

        A node uses HSS arithmetic when its height exceeds h_sw; a non-root
        node compresses its Schur complement when its parent uses HSS
        arithmetic (Algorithm 3.4 with the switching level counted in height
        so that uneven trees are handled node by node)."""
        arith = ["hss" if b.height > h_sw else "dense" for b in self.boxes]
        comp = [b.parent >= 0 and arith[b.parent] == "hss" for b in self.boxes]
        return arith, comp


def build_nd(N, leaf_dofs=32, beta=16, dofs=1):
    """Nested dissection of the N x N node grid of the continuous P1 mesh;
    `dofs` unknowns per node (DOF id = dofs * node + component)."""
    indptr, indices = grid_pattern(N)

    def units_in(b):
        xs = np.arange(b.x0, b.x1)
        ys = np.arange(b.y0, b.y1)
        return (ys[:, None] * N + xs[None, :]).ravel()      # sorted ids

    coords = lambda u: (u % N, u // N)  # noqa: E731
    return _build(N, N * N, 1, dofs, leaf_dofs, beta, units_in, indptr, indices, coords)


def dg_pattern(Nc):
    """Face adjacency of the triangles of the Nc x Nc cell mesh (element id
    2 (j Nc + i) + t, t = 0 lower, 1 upper), including the diagonal: lower
    (i,j) meets upper (i,j), upper (i,j-1) across its south edge and upper
    (i+1,j) across its east edge."""
    ne = 2 * Nc * Nc
    r, c = [np.arange(ne)], [np.arange(ne)]
    j, i = np.meshgrid(np.arange(Nc), np.arange(Nc), indexing="ij")
    i, j = i.ravel(), j.ravel()
    lo = 2 * (j * Nc + i)
    pairs = [(lo, lo + 1)]
    m = j > 0
    pairs.append((lo[m], 2 * ((j[m] - 1) * Nc + i[m]) + 1))
    m = i < Nc - 1
    pairs.append((lo[m], 2 * (j[m] * Nc + i[m] + 1) + 1))
    for a, b in pairs:
        r += [a, b]
        c += [b, a]
    r, c = np.concatenate(r), np.concatenate(c)
    key = np.unique(r * ne + c)
    rows, cols = key // ne, key % ne
    indptr = np.zeros(ne + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    return np.cumsum(indptr), cols


def build_nd_dg(Nc, leaf_dofs=60, beta=60, dofs=6):
    """Nested dissection of the discontinuous mesh (Sec. 3.3, Fig. 5 left):
    boxes are half-open cell ranges of the Nc x Nc cell grid, whole triangles
    are the units (each cell holds two), two triangles are adjacent when they
    share a face, and each triangle carries `dofs` unknowns (6 for P2; DOF id
    = dofs * element + local index).  A box with nx ny 2 dofs <= leaf_dofs is
    a leaf.  Cluster bisection uses the triangle centroids in units of h/3:
    (3i + 2, 3j + 1) for the lower and (3i + 1, 3j + 2) for the upper
    triangle of cell (i, j)."""
    indptr, indices = dg_pattern(Nc)

    def units_in(b):
        xs = np.arange(b.x0, b.x1)
        ys = np.arange(b.y0, b.y1)
        cells = (ys[:, None] * Nc + xs[None, :]).ravel()
        return (2 * cells[:, None] + np.arange(2)[None, :]).ravel()   # sorted ids

    def coords(u):
        cell, t = u // 2, u % 2
        i, j = cell % Nc, cell // Nc
        return 3 * i + 2 - t, 3 * j + 1 + t

    return _build(Nc, 2 * Nc * Nc, 2, dofs, leaf_dofs, beta, units_in, indptr, indices, coords)


def _build(G, n_units, per_cell, dofs, leaf_dofs, beta, units_in, indptr, indices, coords):
    """Shared core: boxes over the G x G grid of nodes (CG) or cells (DG)
    holding per_cell units each; unit adjacency from the CSR pattern."""
    boxes = []

    def rec(x0, x1, y0, y1, depth):
        nx, ny = x1 - x0, y1 - y0
        b = Box(x0, x1, y0, y1, depth=depth)
        if nx * ny * per_cell * dofs > leaf_dofs:
            if nx >= ny:
                xm = x0 + nx // 2
                lo = rec(x0, xm, y0, y1, depth + 1)
                hi = rec(xm, x1, y0, y1, depth + 1)
            else:
                ym = y0 + ny // 2
                lo = rec(x0, x1, y0, ym, depth + 1)
                hi = rec(x0, x1, ym, y1, depth + 1)
            b.lo, b.hi = lo, hi
            b.height = 1 + max(boxes[lo].height, boxes[hi].height)
        boxes.append(b)
        k = len(boxes) - 1
        if b.lo >= 0:
            boxes[b.lo].parent = k
            boxes[b.hi].parent = k
        return k

    rec(0, G, 0, G, 0)

    # Bd(sigma): units of the box with a structural neighbour outside the box
    inbox = np.zeros(n_units, dtype=bool)
    for b in boxes:
        units = units_in(b)
        inbox[units] = True
        cnt = indptr[units + 1] - indptr[units]
        rows = np.repeat(units, cnt)
        first = np.repeat(indptr[units] - np.cumsum(cnt) + cnt, cnt)
        nbr = indices[first + np.arange(cnt.sum())]
        outside = ~inbox[nbr]
        b.bd = np.unique(rows[outside])
        inbox[units] = False
        b._units = np.sort(units)

    # B order (cluster trees) and P0 sizes; needs the parent's Bd
    for k, b in enumerate(boxes):
        if b.parent < 0:
            b.B = np.zeros(0, dtype=np.int64)
            b.p0 = 0
            b.ctree, _ = _cluster_tree([], coords, beta, dofs)
            continue
        pbd = boxes[b.parent].bd
        in_pb = np.isin(b.bd, pbd)
        P0 = b.bd[~in_pb]
        P1 = b.bd[in_pb]
        b.ctree, b.B = _cluster_tree([P0, P1], coords, beta, dofs)
        b.p0 = P0.size

    # I order
    for b in boxes:
        if b.is_leaf:
            b.I = np.setdiff1d(b._units, b.bd)          # sorted unit ids
        else:
            mu, nu = boxes[b.lo], boxes[b.hi]
            b.I = np.concatenate([mu.B[:mu.p0], nu.B[:nu.p0]])
        del b._units

    if dofs > 1:
        _expand_dofs(boxes, dofs)
    perm = np.concatenate([b.I for b in boxes]).astype(np.int64)
    off = 0
    for b in boxes:
        b.offset = off
        off += b.I.size
    n_dof = n_units * dofs
    iperm = np.empty(n_dof, dtype=np.int64)
    iperm[perm] = np.arange(n_dof)
    t = NDTree(N=G, leaf_dofs=leaf_dofs, beta=beta, dofs=dofs, boxes=boxes,
               perm=perm, iperm=iperm)
    return t


def _expand_dofs(boxes, dofs):
    """Node lists -> DOF lists for `dofs` unknowns per node (DOF id =
    dofs * node + component): every node becomes its consecutive components,
    cluster ranges and P0 sizes scale by `dofs`."""
    comp = np.arange(dofs, dtype=np.int64)
    ex = lambda v: (np.asarray(v, dtype=np.int64)[:, None] * dofs + comp[None, :]).ravel()  # noqa: E731
    for b in boxes:
        b.I = ex(b.I)
        b.B = ex(b.B)
        b.p0 = b.p0 * dofs
        ct = b.ctree
        b.ctree = ClusterTree(ct.start * dofs, ct.size * dofs, ct.left, ct.right, ct.level)
