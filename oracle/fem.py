"""P1 continuous Galerkin assembly of the 2D Helmholtz operator (oracle).

Problem (Sec. 4.2, eq. 4.2, with the first-order absorbing condition that
replaces the paper's Dirichlet/Neumann data):

    -lap u - k(x)^2 u = f  in [0,1]^2,     d_n u - i k(x) u = 0  on the boundary,
    k(x) = omega * s(x), s = slowness.

Weak form with the bilinear (not sesquilinear) pairing, so the matrix is
complex symmetric:

    A = K - omega^2 M[s^2] - i omega G[s],

    K_ij    = int grad phi_i . grad phi_j
    M[w]_ij = sum_l w_l int_T phi_l phi_i phi_j          (w interpolated as P1)
    G[s]_ij = sum_l s_l int_boundary phi_l phi_i phi_j   (s interpolated as P1)

Mesh: every grid cell (i,j) is split along its SW-NE diagonal into
{(i,j),(i+1,j),(i+1,j+1)} and {(i,j),(i+1,j+1),(i,j+1)} (the "regular
triangular mesh" of Sec. 4.1).  The load vector of a nodal source f_I is
b = M[1] f_I.

Monomial integrals over barycentric coordinates (exact closed forms):
    int_T  l0^a l1^b l2^c = 2|T| a! b! c! / (a+b+c+2)!
    int_e  l0^a l1^b      =  |e| a! b!    / (a+b+1)!
"""
from math import factorial

import numpy as np
import scipy.sparse as sp

__all__ = ["triangles", "boundary_edges", "assemble_helmholtz", "mass_matrix",
           "stencil_nnz", "element_terms", "assemble_parts", "assemble_elastic",
           "assemble_elastic_parts", "mass_matrix_vec"]


def triangles(N):
    """(nt, 3) int64 node ids; cell (i,j) gives two triangles (SW-NE diagonal)."""
    i, j = np.meshgrid(np.arange(N - 1), np.arange(N - 1), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    a = j * N + i
    b = j * N + i + 1
    c = (j + 1) * N + i + 1
    d = (j + 1) * N + i
    t1 = np.stack([a, b, c], axis=1)
    t2 = np.stack([a, c, d], axis=1)
    out = np.empty((2 * t1.shape[0], 3), dtype=np.int64)
    out[0::2] = t1
    out[1::2] = t2
    return out


def boundary_edges(N):
    """(ne, 2) int64 node ids of the 4(N-1) boundary edges."""
    k = np.arange(N - 1)
    south = np.stack([k, k + 1], axis=1)
    north = np.stack([(N - 1) * N + k, (N - 1) * N + k + 1], axis=1)
    west = np.stack([k * N, (k + 1) * N], axis=1)
    east = np.stack([k * N + N - 1, (k + 1) * N + N - 1], axis=1)
    return np.concatenate([south, east, north, west], axis=0)


def _tri_int(a, b, c):
    """int_T l0^a l1^b l2^c divided by 2|T|."""
    return factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 2)


def _edge_int(a, b):
    """int_e l0^a l1^b divided by |e|."""
    return factorial(a) * factorial(b) / factorial(a + b + 1)


# T3[l, i, j] = int_T l_l l_i l_j / (2|T|);  E3[l, i, j] likewise on an edge.
_T3 = np.zeros((3, 3, 3))
for _l in range(3):
    for _i in range(3):
        for _j in range(3):
            e = [0, 0, 0]
            e[_l] += 1
            e[_i] += 1
            e[_j] += 1
            _T3[_l, _i, _j] = _tri_int(*e)
_T2 = np.zeros((3, 3))
for _i in range(3):
    for _j in range(3):
        e = [0, 0, 0]
        e[_i] += 1
        e[_j] += 1
        _T2[_i, _j] = _tri_int(*e)
_E3 = np.zeros((2, 2, 2))
for _l in range(2):
    for _i in range(2):
        for _j in range(2):
            e = [0, 0]
            e[_l] += 1
            e[_i] += 1
            e[_j] += 1
            _E3[_l, _i, _j] = _edge_int(*e)


def element_terms(N):
    """Per-triangle geometry: (tris, area, K_local (nt,3,3)) for the mesh."""
    h = 1.0 / (N - 1)
    tris = triangles(N)
    xy = np.stack([(tris % N) * h, (tris // N) * h], axis=-1)   # (nt, 3, 2)
    e1 = xy[:, 1] - xy[:, 0]
    e2 = xy[:, 2] - xy[:, 0]
    det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    area = 0.5 * np.abs(det)
    # gradient of barycentric l_a = rot(opposite edge) / (2|T|) (signed)
    grads = np.empty((tris.shape[0], 3, 2))
    for a in range(3):
        p = xy[:, (a + 1) % 3]
        q = xy[:, (a + 2) % 3]
        d = q - p
        grads[:, a, 0] = d[:, 1] / det
        grads[:, a, 1] = -d[:, 0] / det
    K = area[:, None, None] * np.einsum("tad,tbd->tab", grads, grads)
    return tris, area, K


def assemble_parts(N, s):
    """Element contributions accumulated into the unique unordered node pairs.

    Returns (rows, cols, vals) with rows <= cols and vals a dict of float64
    arrays for K, M[s^2] ("M2"), M[1] ("M1") and G[s] ("G").  Each element adds
    its local entries (a, b) with a <= b once, in a fixed order (element order,
    then local pair order), so mirroring the result gives a bitwise symmetric
    matrix."""
    s = np.asarray(s, dtype=np.float64)
    tris, area, Kl = element_terms(N)
    w = s[tris] ** 2                                            # (nt, 3)
    Ml = 2.0 * area[:, None, None] * np.einsum("tl,lij->tij", w, _T3)
    M1 = 2.0 * area[:, None, None] * _T2[None, :, :]
    edges = boundary_edges(N)
    h = 1.0 / (N - 1)
    Gl = h * np.einsum("el,lij->eij", s[edges], _E3)

    n = N * N
    ta, tb = np.triu_indices(3)
    ea, eb = np.triu_indices(2)
    r = np.concatenate([tris[:, ta].ravel(), edges[:, ea].ravel()])
    c = np.concatenate([tris[:, tb].ravel(), edges[:, eb].ravel()])
    lo = np.minimum(r, c)
    hi = np.maximum(r, c)
    uniq, inv = np.unique(lo * n + hi, return_inverse=True)
    nt = tris.shape[0] * ta.size
    vals = {}
    for name, loc_t, loc_e in (("K", Kl, None), ("M2", Ml, None),
                               ("M1", M1, None), ("G", None, Gl)):
        acc = np.zeros(uniq.size)
        if loc_t is not None:
            np.add.at(acc, inv[:nt], loc_t[:, ta, tb].ravel())
        if loc_e is not None:
            np.add.at(acc, inv[nt:], loc_e[:, ea, eb].ravel())
        vals[name] = acc
    return uniq // n, uniq % n, vals


def _mirror_csr(n, rows, cols, v):
    off = rows != cols
    R = np.concatenate([rows, cols[off]])
    C = np.concatenate([cols, rows[off]])
    V = np.concatenate([v, v[off]])
    A = sp.csr_matrix((V, (R, C)), shape=(n, n))
    A.sort_indices()
    return A


def assemble_helmholtz(N, omega, s=None):
    """A = K - omega^2 M[s^2] - i omega G[s] as a scipy CSR complex128 matrix
    with sorted column indices, on the natural node numbering j*N + i."""
    n = N * N
    if s is None:
        s = np.ones(n)
    rows, cols, v = assemble_parts(N, s)
    val = v["K"] - omega * omega * v["M2"] - 1j * omega * v["G"]
    return _mirror_csr(n, rows, cols, val.astype(np.complex128))


def mass_matrix(N):
    """Plain mass matrix M[1] (real CSR); the load of a nodal source is M f."""
    n = N * N
    rows, cols, v = assemble_parts(N, np.ones(n))
    return _mirror_csr(n, rows, cols, v["M1"])


def stencil_nnz(N):
    """Structural nonzeros of the 7-point P1 stencil on this mesh."""
    return N * N + 2 * (2 * N * (N - 1) + (N - 1) ** 2)


# ---------------------------------------------------------------- elastic
#
# Time-harmonic linear elasticity, P1 vector elements on the same mesh
# (the elastic workload of the paper's numerical section):
#
#     -div sigma(u) - omega^2 rho u = f,   sigma(u) = lam (div u) I + mu (grad u + grad u^T),
#
# with the first-order absorbing (Lysmer-Kuhlemeyer) traction
# sigma(u) n = i omega rho (c_p (u.n) n + c_s (u.t) t) on the boundary,
# c_p = sqrt((lam + 2 mu) / rho), c_s = sqrt(mu / rho).  Bilinear pairing:
#
#     A = K[lam, mu] - omega^2 M[rho] - i omega C,
#
#     K_(a,i),(b,j) = int lam d_i phi_a d_j phi_b + mu (delta_ij grad phi_a . grad phi_b
#                                                       + d_j phi_a d_i phi_b)
#     M[rho]_(a,i),(b,j) = delta_ij sum_l rho_l int phi_l phi_a phi_b
#     C_(a,i),(b,j) = sum_l int_e phi_l phi_a phi_b (zp_l n_i n_j + zs_l t_i t_j),
#                     zp = rho c_p, zs = rho c_s (nodal values interpolated as P1)
#
# lam, mu enter K through their element means (P1 interpolation, constant
# gradients).  DOF id = 2 * node + component.

def _edge_normals(N):
    """Per boundary edge (same order as boundary_edges): n n^T and t t^T."""
    k = N - 1
    nn = np.zeros((4 * k, 2, 2))
    tt = np.zeros((4 * k, 2, 2))
    nn[:k, 1, 1] = 1.0          # south, n = (0, -1)
    tt[:k, 0, 0] = 1.0
    nn[k:2 * k, 0, 0] = 1.0     # east, n = (1, 0)
    tt[k:2 * k, 1, 1] = 1.0
    nn[2 * k:3 * k, 1, 1] = 1.0  # north
    tt[2 * k:3 * k, 0, 0] = 1.0
    nn[3 * k:, 0, 0] = 1.0       # west
    tt[3 * k:, 1, 1] = 1.0
    return nn, tt


def assemble_elastic_parts(N, lam, mu, rho):
    """Unordered DOF pairs (rows <= cols) with float64 values of K, M[rho],
    M[1] (plain vector mass) and C; each element adds its local pairs once in
    a fixed order, so mirroring gives a bitwise symmetric matrix."""
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    h = 1.0 / (N - 1)
    tris = triangles(N)
    xy = np.stack([(tris % N) * h, (tris // N) * h], axis=-1)
    e1 = xy[:, 1] - xy[:, 0]
    e2 = xy[:, 2] - xy[:, 0]
    det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    area = 0.5 * np.abs(det)
    g = np.empty((tris.shape[0], 3, 2))
    for a in range(3):
        d = xy[:, (a + 2) % 3] - xy[:, (a + 1) % 3]
        g[:, a, 0] = d[:, 1] / det
        g[:, a, 1] = -d[:, 0] / det
    lam_t = lam[tris].mean(axis=1) * area
    mu_t = mu[tris].mean(axis=1) * area
    eye = np.eye(2)
    # Kl[t, a, i, b, j]
    gg = np.einsum("tad,tbd->tab", g, g)
    Kl = (lam_t[:, None, None, None, None] * np.einsum("tai,tbj->taibj", g, g)
          + mu_t[:, None, None, None, None] * (np.einsum("tab,ij->taibj", gg, eye)
                                               + np.einsum("taj,tbi->taibj", g, g)))
    Ms = 2.0 * area[:, None, None] * np.einsum("tl,lij->tij", rho[tris], _T3)
    M1s = 2.0 * area[:, None, None] * _T2[None, :, :]
    Ml = np.einsum("tab,ij->taibj", Ms, eye)
    M1l = np.einsum("tab,ij->taibj", M1s, eye)
    edges = boundary_edges(N)
    zp = np.sqrt(rho * (lam + 2.0 * mu))
    zs = np.sqrt(rho * mu)
    nn, tt = _edge_normals(N)
    Ep = h * np.einsum("el,lab->eab", zp[edges], _E3)
    Es = h * np.einsum("el,lab->eab", zs[edges], _E3)
    Cl = (np.einsum("eab,eij->eaibj", Ep, nn) + np.einsum("eab,eij->eaibj", Es, tt))

    n = 2 * N * N
    # local DOF lists: triangle (3 nodes x 2) and edge (2 nodes x 2)
    tdof = (2 * tris[:, :, None] + np.arange(2)[None, None, :]).reshape(-1, 6)
    edof = (2 * edges[:, :, None] + np.arange(2)[None, None, :]).reshape(-1, 4)
    ta, tb = np.triu_indices(6)
    ea, eb = np.triu_indices(4)
    r = np.concatenate([tdof[:, ta].ravel(), edof[:, ea].ravel()])
    c = np.concatenate([tdof[:, tb].ravel(), edof[:, eb].ravel()])
    lo = np.minimum(r, c)
    hi = np.maximum(r, c)
    uniq, inv = np.unique(lo * n + hi, return_inverse=True)
    nt = tris.shape[0] * ta.size
    vals = {}
    for name, loc_t, loc_e in (("K", Kl, None), ("M", Ml, None), ("M1", M1l, None),
                               ("C", None, Cl)):
        acc = np.zeros(uniq.size)
        if loc_t is not None:
            np.add.at(acc, inv[:nt], loc_t.reshape(-1, 6, 6)[:, ta, tb].ravel())
        if loc_e is not None:
            np.add.at(acc, inv[nt:], loc_e.reshape(-1, 4, 4)[:, ea, eb].ravel())
        vals[name] = acc
    return uniq // n, uniq % n, vals


def assemble_elastic(N, omega, lam, mu, rho):
    """A = K - omega^2 M[rho] - i omega C (complex128 CSR, sorted columns) on
    DOF ids 2 * node + component.  Structural zeros of the 14-entry block
    pattern are kept as explicit entries."""
    n = 2 * N * N
    rows, cols, v = assemble_elastic_parts(N, lam, mu, rho)
    val = v["K"] - omega * omega * v["M"] - 1j * omega * v["C"]
    return _mirror_csr(n, rows, cols, val.astype(np.complex128))


def mass_matrix_vec(N):
    """Plain vector mass matrix (DOF ids 2 * node + component)."""
    n = 2 * N * N
    rows, cols, v = assemble_elastic_parts(N, np.ones(N * N), np.ones(N * N), np.ones(N * N))
    return _mirror_csr(n, rows, cols, v["M1"])
