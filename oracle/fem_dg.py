"""Symmetric interior-penalty DG discretizations of the Helmholtz problem
with P1 or P2 elements (oracle; test infrastructure only).

The paper's IPDG runs (Sec. 4.1-4.2 and the scaling study of Sec. 4.6) use
interior-penalty discontinuous Galerkin on a regular triangular mesh.  This
module writes out the symmetric variant for

    -lap u - k(x)^2 u = f  on [0,1]^2,   k = omega s(x),

as the complex-symmetric bilinear form (no conjugation)

    a(u, v) = sum_T int_T (grad u . grad v - k^2 u v)
            + sum_{interior F} ( - int_F {grad u . n}[v] - int_F {grad v . n}[u]
                                 + tau_F int_F [u][v] )
            + boundary terms,

with [w] = w+ - w-, {w} = (w+ + w-)/2, n the unit normal from + to -, and
tau_F = 10 p^2 / |F| (p the polynomial degree, |F| the face length).  The
boundary terms are either the first-order absorbing condition
d_n u - i k u = 0,

            - i sum_{boundary F} int_F k u v ,

or the homogeneous Dirichlet condition u = 0 of Sec. 4.1-4.2 and 4.6, imposed
as in the interior with the outside value zero (n the outward normal):

            sum_{boundary F} ( - int_F (grad u . n) v - int_F (grad v . n) u
                               + tau_F int_F u v ).

k^2 is the P1 interpolant of the nodal omega^2 s^2 inside each triangle, k on
a boundary face the P1 interpolant of omega s.

Mesh: Nc x Nc cells of side h = 1/Nc; cell (i, j) holds the lower triangle
t = 0 with vertices (i,j), (i+1,j), (i+1,j+1) and the upper triangle t = 1
with (i,j), (i+1,j+1), (i,j+1) (grid vertices, counter-clockwise).  Element
id e = 2 (j Nc + i) + t.  Each element carries the nodal Lagrange functions
of degree p: the three vertices in that order, then (p = 2) the midpoints of
edges (v0,v1), (v1,v2), (v2,v0).  DOF id = nb e + a with nb = 3 (P1) or 6
(P2).  Faces: f = 0 is (v0,v1), f = 1 is (v1,v2), f = 2 is (v2,v0).

Quadrature: collapsed (Duffy) 4 x 4 Gauss-Legendre on triangles (exact to
degree 6), 4-point Gauss-Legendre on faces (degree 7).
"""
import numpy as np
import scipy.sparse as sp

__all__ = ["P", "PENALTY", "nbasis", "elements", "dof_coords", "faces", "basis",
           "assemble_dg_parts", "assemble_dg", "mass_matrix_dg", "dg_nnz"]

P = 2            # default polynomial degree
PENALTY = 10.0


def nbasis(deg):
    """Nodal functions per triangle: 3 (P1) or 6 (P2)."""
    assert deg in (1, 2)
    return (deg + 1) * (deg + 2) // 2

_T4, _W4 = np.polynomial.legendre.leggauss(4)
_T4 = (_T4 + 1.0) / 2.0
_W4 = _W4 / 2.0


def elements(Nc):
    """Vertex coordinates (2 Nc^2, 3, 2) and vertex grid ids (2 Nc^2, 3)."""
    h = 1.0 / Nc
    j, i = np.meshgrid(np.arange(Nc), np.arange(Nc), indexing="ij")
    i, j = i.ravel(), j.ravel()
    Nv = Nc + 1
    vid = np.empty((2 * Nc * Nc, 3), dtype=np.int64)
    vid[0::2] = np.stack([j * Nv + i, j * Nv + i + 1, (j + 1) * Nv + i + 1], axis=1)
    vid[1::2] = np.stack([j * Nv + i, (j + 1) * Nv + i + 1, (j + 1) * Nv + i], axis=1)
    xy = np.stack([(vid % Nv) * h, (vid // Nv) * h], axis=-1)
    return xy, vid


def _local_nodes(V, deg=P):
    """Node coordinates of elements with vertices V (..., 3, 2)."""
    if deg == 1:
        return V
    mid = np.stack([(V[..., 0, :] + V[..., 1, :]) / 2, (V[..., 1, :] + V[..., 2, :]) / 2,
                    (V[..., 2, :] + V[..., 0, :]) / 2], axis=-2)
    return np.concatenate([V, mid], axis=-2)


def dof_coords(Nc, deg=P):
    """(2 Nc^2 nb, 2) coordinates of the DOF nodes."""
    V, _ = elements(Nc)
    return _local_nodes(V, deg).reshape(-1, 2)


def _bary(V, p):
    """Barycentric coordinates of points p (E, Q, 2) in triangles V (E, 3, 2),
    and their constant gradients (E, 3, 2)."""
    det = ((V[:, 1, 0] - V[:, 0, 0]) * (V[:, 2, 1] - V[:, 0, 1])
           - (V[:, 1, 1] - V[:, 0, 1]) * (V[:, 2, 0] - V[:, 0, 0]))
    lam = np.empty(p.shape[:2] + (3,))
    grad = np.empty((V.shape[0], 3, 2))
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        # twice the signed area of (p, v_b, v_c) over twice the element area
        ax = V[:, b, None, 0] - p[..., 0]
        ay = V[:, b, None, 1] - p[..., 1]
        bx = V[:, c, None, 0] - p[..., 0]
        by = V[:, c, None, 1] - p[..., 1]
        lam[..., a] = (ax * by - ay * bx) / det[:, None]
        grad[:, a, 0] = (V[:, b, 1] - V[:, c, 1]) / det
        grad[:, a, 1] = (V[:, c, 0] - V[:, b, 0]) / det
    return lam, grad, det


_EDGES = ((0, 1), (1, 2), (2, 0))


def basis(V, p, deg=P):
    """Values (E, Q, nb) and gradients (E, Q, nb, 2) at points p (E, Q, 2) of
    the degree-deg nodal functions: the barycentric coordinates for P1; for
    P2 lam_a (2 lam_a - 1) at the vertices and 4 lam_a lam_b at the edge
    midpoints."""
    lam, g, _ = _bary(V, p)
    if deg == 1:
        return lam.copy(), np.broadcast_to(g[:, None, :, :], lam.shape + (2,)).copy()
    phi = np.empty(lam.shape[:2] + (6,))
    dphi = np.empty(lam.shape[:2] + (6, 2))
    for a in range(3):
        phi[..., a] = lam[..., a] * (2.0 * lam[..., a] - 1.0)
        dphi[..., a, :] = (4.0 * lam[..., a, None] - 1.0) * g[:, None, a, :]
    for m, (a, b) in enumerate(_EDGES):
        phi[..., 3 + m] = 4.0 * lam[..., a] * lam[..., b]
        dphi[..., 3 + m, :] = 4.0 * (lam[..., b, None] * g[:, None, a, :]
                                     + lam[..., a, None] * g[:, None, b, :])
    return phi, dphi


def _tri_quad(V):
    """Collapsed Gauss points (E, 16, 2), their weights (E, 16) (area
    included) and barycentric coordinates (16, 3)."""
    u, v = np.meshgrid(_T4, _T4, indexing="ij")
    wu, wv = np.meshgrid(_W4, _W4, indexing="ij")
    xi = u.ravel()
    eta = (v * (1.0 - u)).ravel()
    w = (wu * wv * (1.0 - u)).ravel()
    e1 = V[:, 1] - V[:, 0]
    e2 = V[:, 2] - V[:, 0]
    det = np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    pts = V[:, None, 0] + xi[None, :, None] * e1[:, None] + eta[None, :, None] * e2[:, None]
    lam = np.stack([1.0 - xi - eta, xi, eta], axis=1)
    return pts, w[None, :] * det[:, None], lam


def faces(Nc):
    """Interior faces (plus element, plus local face, minus element, minus
    local face) with the plus element the lower id, and boundary faces
    (element, local face)."""
    inner, bnd = [], []
    for j in range(Nc):
        for i in range(Nc):
            lo = 2 * (j * Nc + i)
            up = lo + 1
            inner.append((lo, 2, up, 0))                       # cell diagonal
            if j > 0:
                inner.append((2 * ((j - 1) * Nc + i) + 1, 1, lo, 0))   # south edge
            else:
                bnd.append((lo, 0))
            if i < Nc - 1:
                inner.append((lo, 1, 2 * (j * Nc + i + 1) + 1, 2))    # east edge
            else:
                bnd.append((lo, 1))
            if j == Nc - 1:
                bnd.append((up, 1))                            # north
            if i == 0:
                bnd.append((up, 2))                            # west
    inner = np.array(inner, dtype=np.int64).reshape(-1, 4)
    for r in range(inner.shape[0]):
        if inner[r, 0] > inner[r, 2]:
            inner[r] = inner[r, [2, 3, 0, 1]]
    return inner, np.array(bnd, dtype=np.int64).reshape(-1, 2)


def _face_points(V, f):
    """Gauss points (E, 4, 2), weights times length (E, 4), unit outward
    normals (E, 2) and lengths (E,) of local faces f of elements V."""
    a = np.array([_EDGES[k][0] for k in f])
    b = np.array([_EDGES[k][1] for k in f])
    E = np.arange(V.shape[0])
    ps, pe = V[E, a], V[E, b]
    d = pe - ps
    L = np.hypot(d[:, 0], d[:, 1])
    pts = ps[:, None, :] + _T4[None, :, None] * d[:, None, :]
    nrm = np.stack([d[:, 1], -d[:, 0]], axis=1) / L[:, None]
    return pts, _W4[None, :] * L[:, None], nrm, L


def assemble_dg_parts(Nc, omega, s_vertex, deg=P, bc="absorbing"):
    """Unordered DOF pairs (rows <= cols) with the values of A and of the
    plain DG mass matrix; each pair accumulates its contributions in a fixed
    order, so mirroring yields a bitwise symmetric matrix.  deg: 1 or 2;
    bc: "absorbing" or "dirichlet"."""
    assert bc in ("absorbing", "dirichlet")
    nb = nbasis(deg)
    s = np.asarray(s_vertex, dtype=np.float64)
    V, vid = elements(Nc)
    ne = V.shape[0]
    rows, cols, vals, mvals = [], [], [], []
    ia, ib = np.triu_indices(nb)

    # volume terms
    pts, w, lam = _tri_quad(V)
    phi, dphi = basis(V, pts, deg)
    k2 = omega * omega * (lam[None, :, :] * (s[vid] ** 2)[:, None, :]).sum(axis=2)
    Kl = np.einsum("eq,eqad,eqbd->eab", w, dphi, dphi)
    Ml = np.einsum("eq,eqa,eqb->eab", w * k2, phi, phi)
    M1 = np.einsum("eq,eqa,eqb->eab", w, phi, phi)
    dof = nb * np.arange(ne)[:, None] + np.arange(nb)[None, :]
    rows.append(dof[:, ia].ravel())
    cols.append(dof[:, ib].ravel())
    vals.append((Kl - Ml)[:, ia, ib].ravel().astype(np.complex128))
    mvals.append(M1[:, ia, ib].ravel())

    # interior faces
    inner, bnd = faces(Nc)
    ep, fp, em, _ = inner.T
    fpts, fw, nrm, L = _face_points(V[ep], fp)
    tau = PENALTY * deg * deg / L
    php, dpp = basis(V[ep], fpts, deg)
    phm, dpm = basis(V[em], fpts, deg)
    dnp = np.einsum("eqad,ed->eqa", dpp, nrm)
    dnm = np.einsum("eqad,ed->eqa", dpm, nrm)
    # block (row side, column side): sides + (sign +1) and - (sign -1)
    for rs, cs in ((0, 0), (1, 1), (0, 1)):
        pr, dr, sr = (php, dnp, 1.0) if rs == 0 else (phm, dnm, -1.0)
        pc, dc, sc = (php, dnp, 1.0) if cs == 0 else (phm, dnm, -1.0)
        blk = (-0.5 * sr * np.einsum("eq,eqb,eqa->eab", fw, dc, pr)
               - 0.5 * sc * np.einsum("eq,eqa,eqb->eab", fw, dr, pc)
               + (sr * sc) * tau[:, None, None] * np.einsum("eq,eqa,eqb->eab", fw, pr, pc))
        er = ep if rs == 0 else em
        ec = ep if cs == 0 else em
        R = nb * er[:, None, None] + np.arange(nb)[None, :, None]
        Cc = nb * ec[:, None, None] + np.arange(nb)[None, None, :]
        R = np.broadcast_to(R, blk.shape)
        Cc = np.broadcast_to(Cc, blk.shape)
        keep = R <= Cc
        rows.append(R[keep])
        cols.append(Cc[keep])
        vals.append(blk[keep].astype(np.complex128))
        mvals.append(np.zeros(int(keep.sum())))

    # boundary faces: absorbing, or Dirichlet with the outside value zero
    eb, fb = bnd.T
    bpts, bw, bn, bL = _face_points(V[eb], fb)
    phb, dphb = basis(V[eb], bpts, deg)
    if bc == "absorbing":
        lam_b, _, _ = _bary(V[eb], bpts)
        kb = omega * (lam_b * s[vid[eb]][:, None, :]).sum(axis=2)
        Gl = -1j * np.einsum("eq,eqa,eqb->eab", bw * kb, phb, phb)
    else:
        dnb = np.einsum("eqad,ed->eqa", dphb, bn)
        taub = PENALTY * deg * deg / bL
        Gl = (-np.einsum("eq,eqb,eqa->eab", bw, dnb, phb)
              - np.einsum("eq,eqa,eqb->eab", bw, dnb, phb)
              + taub[:, None, None] * np.einsum("eq,eqa,eqb->eab", bw, phb, phb))
    dofb = nb * eb[:, None] + np.arange(nb)[None, :]
    rows.append(dofb[:, ia].ravel())
    cols.append(dofb[:, ib].ravel())
    vals.append(Gl[:, ia, ib].ravel().astype(np.complex128))
    mvals.append(np.zeros(ia.size * eb.size))

    r = np.concatenate(rows)
    c = np.concatenate(cols)
    n = nb * ne
    uniq, inv = np.unique(r * n + c, return_inverse=True)
    acc = np.zeros(uniq.size, dtype=np.complex128)
    np.add.at(acc, inv, np.concatenate(vals))
    macc = np.zeros(uniq.size)
    np.add.at(macc, inv, np.concatenate(mvals))
    return uniq // n, uniq % n, acc, macc


def _mirror(n, rows, cols, v):
    off = rows != cols
    R = np.concatenate([rows, cols[off]])
    C = np.concatenate([cols, rows[off]])
    Vv = np.concatenate([v, v[off]])
    return sp.csr_matrix((Vv, (R, C)), shape=(n, n))


def assemble_dg(Nc, omega, s_vertex=None, deg=P, bc="absorbing"):
    """A (complex128 CSR, sorted columns) on DOFs nb e + a.  Structural zeros
    of the element-face block pattern are kept as explicit entries.
    s_vertex: nodal slowness on the (Nc+1)^2 vertex grid (default 1)."""
    if s_vertex is None:
        s_vertex = np.ones((Nc + 1) ** 2)
    rows, cols, v, _ = assemble_dg_parts(Nc, omega, s_vertex, deg, bc)
    A = _mirror(2 * Nc * Nc * nbasis(deg), rows, cols, v)
    A.sort_indices()
    return A


def mass_matrix_dg(Nc, deg=P):
    """Block-diagonal mass matrix of the nodal basis (the load b = M f of
    nodal samples)."""
    rows, cols, _, m = assemble_dg_parts(Nc, 0.0, np.ones((Nc + 1) ** 2), deg)
    M = _mirror(2 * Nc * Nc * nbasis(deg), rows, cols, m)
    M.eliminate_zeros()
    return M


def dg_nnz(Nc, deg=P):
    """Entries of the element-face block pattern: nb^2 per element self block
    and per face-neighbour block."""
    nb = nbasis(deg)
    return nb * nb * (2 * Nc * Nc + 2 * (3 * Nc * Nc - 2 * Nc))
