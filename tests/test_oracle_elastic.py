"""Pins of the oracle's P1 elastic assembly (the time-harmonic elastic
operator of Sec. 4, eq. 4.6, with a first-order absorbing traction) against
facts that do not come from the oracle: rigid motions in the kernel of the
stiffness, exact energies of affine fields, exact mass and boundary integrals
by Gauss quadrature, and the second-order convergence of manufactured P- and
S-plane waves."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem

NORMALS = np.array([[0.0, -1.0], [1.0, 0.0], [0.0, 1.0], [-1.0, 0.0]])  # S, E, N, W


def _xy(N):
    h = 1.0 / (N - 1)
    i = np.arange(N) * h
    return np.tile(i, N), np.repeat(i, N)


def _vec(ux, uy):
    u = np.empty(2 * ux.size, dtype=np.result_type(ux, uy))
    u[0::2], u[1::2] = ux, uy
    return u


def _parts(N, lam, mu, rho):
    import scipy.sparse as sp
    r, c, v = fem.assemble_elastic_parts(N, lam, mu, rho)
    n = 2 * N * N
    out = {}
    for k, val in v.items():
        M = sp.coo_matrix((val, (r, c)), shape=(n, n)).tocsr()
        out[k] = M + sp.triu(M, 1).T
    return out


@pytest.mark.parametrize("N", [2, 5, 17])
def test_pattern_and_bitwise_symmetry(N):
    rng = np.random.default_rng(N)
    lam, mu = 1 + rng.random(N * N), 0.5 + rng.random(N * N)
    A = fem.assemble_elastic(N, 7.0, lam, mu, 1 + rng.random(N * N))
    assert A.nnz == 4 * fem.stencil_nnz(N)          # 2x2 blocks of the 7-point stencil
    assert (A != A.T).nnz == 0
    for r in range(A.shape[0]):
        assert np.all(np.diff(A.indices[A.indptr[r]:A.indptr[r + 1]]) > 0)


def test_rigid_motions_in_kernel():
    """Translations and the infinitesimal rotation (-y, x) have zero strain,
    so K maps them to zero for any Lame fields."""
    N = 13
    rng = np.random.default_rng(0)
    K = _parts(N, 1 + 3 * rng.random(N * N), 0.5 + rng.random(N * N), np.ones(N * N))["K"]
    x, y = _xy(N)
    for u in (_vec(np.ones(N * N), np.zeros(N * N)), _vec(np.zeros(N * N), np.ones(N * N)),
              _vec(-y, x)):
        assert np.abs(K @ u).max() < 1e-12


def test_affine_energies_exact():
    """For constant lam, mu and affine u, v (exact in P1):
    u.K v = lam div u div v + 2 mu eps(u):eps(v) over the unit square."""
    N = 9
    lam0, mu0 = 1.7, 0.6
    K = _parts(N, np.full(N * N, lam0), np.full(N * N, mu0), np.ones(N * N))["K"]
    x, y = _xy(N)
    rng = np.random.default_rng(1)
    for _ in range(4):
        Gu, Gv = rng.standard_normal((2, 2)), rng.standard_normal((2, 2))
        u = _vec(Gu[0, 0] * x + Gu[0, 1] * y + 0.3, Gu[1, 0] * x + Gu[1, 1] * y)
        v = _vec(Gv[0, 0] * x + Gv[0, 1] * y, Gv[1, 0] * x + Gv[1, 1] * y - 1.1)
        eu, ev = (Gu + Gu.T) / 2, (Gv + Gv.T) / 2
        ref = lam0 * np.trace(Gu) * np.trace(Gv) + 2 * mu0 * np.sum(eu * ev)
        assert u @ (K @ v) == pytest.approx(ref, rel=1e-12, abs=1e-12)


def _gauss_square(f, q=4):
    t, w = np.polynomial.legendre.leggauss(q)
    t, w = (t + 1) / 2, w / 2
    X, Y = np.meshgrid(t, t, indexing="ij")
    return np.sum(np.outer(w, w) * f(X, Y))


def test_mass_exact_for_affine_density():
    """u.M[rho] v = int rho u.v for affine rho, u, v (all exact in P1),
    integrated by tensor Gauss quadrature; components do not couple."""
    N = 7
    x, y = _xy(N)
    rho_f = lambda X, Y: 1.2 + 0.5 * X - 0.3 * Y  # noqa: E731
    P = _parts(N, np.ones(N * N), np.ones(N * N), rho_f(x, y))
    ux = lambda X, Y: 0.4 + X - 2 * Y  # noqa: E731
    uy = lambda X, Y: -1 + 0.5 * X + Y  # noqa: E731
    vx = lambda X, Y: 2 - X  # noqa: E731
    vy = lambda X, Y: X + 3 * Y  # noqa: E731
    u, v = _vec(ux(x, y), uy(x, y)), _vec(vx(x, y), vy(x, y))
    ref = _gauss_square(lambda X, Y: rho_f(X, Y) * (ux(X, Y) * vx(X, Y) + uy(X, Y) * vy(X, Y)))
    assert u @ (P["M"] @ v) == pytest.approx(ref, rel=1e-13)
    ref1 = _gauss_square(lambda X, Y: ux(X, Y) * vx(X, Y) + uy(X, Y) * vy(X, Y))
    assert u @ (P["M1"] @ v) == pytest.approx(ref1, rel=1e-13)
    ex = _vec(np.ones(N * N), np.zeros(N * N))
    ey = _vec(np.zeros(N * N), np.ones(N * N))
    assert abs(ex @ (P["M"] @ ey)) < 1e-15


def test_boundary_traction_exact():
    """u.C v = sum over sides of int zp (u.n)(v.n) + zs (u.t)(v.t) for
    constant impedances and affine u, v (quadratic integrands, 3-point Gauss
    per side)."""
    N = 6
    lam0, mu0, rho0 = 2.0, 0.7, 1.3
    P = _parts(N, np.full(N * N, lam0), np.full(N * N, mu0), np.full(N * N, rho0))
    zp, zs = np.sqrt(rho0 * (lam0 + 2 * mu0)), np.sqrt(rho0 * mu0)
    x, y = _xy(N)
    Gu, Gv = np.array([[1.0, -0.5], [0.3, 2.0]]), np.array([[-1.0, 0.2], [0.7, 0.4]])
    cu, cv = np.array([0.1, -0.4]), np.array([1.0, 0.5])
    uf = lambda X, Y: Gu @ np.stack([X, Y]) + cu[:, None]  # noqa: E731
    vf = lambda X, Y: Gv @ np.stack([X, Y]) + cv[:, None]  # noqa: E731
    u = _vec(*uf(x, y))
    v = _vec(*vf(x, y))
    t, w = np.polynomial.legendre.leggauss(3)
    t, w = (t + 1) / 2, w / 2
    sides = [(t, 0 * t), (1 + 0 * t, t), (t, 1 + 0 * t), (0 * t, t)]
    ref = 0.0
    for (X, Y), n in zip(sides, NORMALS):
        tg = np.array([-n[1], n[0]])
        U, V = uf(X, Y), vf(X, Y)
        ref += np.sum(w * (zp * (n @ U) * (n @ V) + zs * (tg @ U) * (tg @ V)))
    assert u @ (P["C"] @ v) == pytest.approx(ref, rel=1e-13)


def _plane_wave_error(N, omega, theta, kind, lam0=2.0, mu0=0.8, rho0=1.0):
    """Nodal RMS error of the P1 solution for u = a exp(i k d.x): P wave
    (a = d, k = omega / c_p) or S wave (a = d rotated by 90 degrees,
    k = omega / c_s); traction data g = sigma(u) n - i omega Z u on every
    side, b_i = int_boundary g.phi_i by 4-point Gauss per edge."""
    h = 1.0 / (N - 1)
    cp, cs = np.sqrt((lam0 + 2 * mu0) / rho0), np.sqrt(mu0 / rho0)
    zp, zs = rho0 * cp, rho0 * cs
    d = np.array([np.cos(theta), np.sin(theta)])
    a = d if kind == "p" else np.array([-d[1], d[0]])
    k = omega / (cp if kind == "p" else cs)
    G = 1j * k * np.outer(a, d)                       # grad u / e
    sig = lam0 * np.trace(G) * np.eye(2) + mu0 * (G + G.T)

    def u_at(X, Y):
        return a[:, None] * np.exp(1j * k * (d[0] * X + d[1] * Y))[None, :]

    x, y = _xy(N)
    u = _vec(*u_at(x, y))
    nn = N * N
    A = fem.assemble_elastic(N, omega, np.full(nn, lam0), np.full(nn, mu0), np.full(nn, rho0))
    b = np.zeros(2 * nn, dtype=complex)
    edges = fem.boundary_edges(N)
    normals = np.repeat(NORMALS, N - 1, axis=0)
    t, w = np.polynomial.legendre.leggauss(4)
    t, w = (t + 1) / 2, w / 2
    for (p, q), n in zip(edges, normals):
        tg = np.array([-n[1], n[0]])
        X = x[p] + t * (x[q] - x[p])
        Y = y[p] + t * (y[q] - y[p])
        U = u_at(X, Y)
        e = np.exp(1j * k * (d[0] * X + d[1] * Y))
        g = (sig @ n)[:, None] * e[None, :] - 1j * omega * (
            zp * np.outer(n, n @ U) + zs * np.outer(tg, tg @ U))
        for node, phi in ((p, 1 - t), (q, t)):
            b[2 * node:2 * node + 2] += h * (g * (w * phi)[None, :]).sum(axis=1)
    uh = spla.spsolve(A.tocsc(), b)
    return np.sqrt(np.mean(np.abs(uh - u) ** 2))


@pytest.mark.parametrize("kind", ["p", "s"])
def test_plane_wave_second_order(kind):
    errs = [_plane_wave_error(N, 6.0, np.pi / 5, kind) for N in (17, 33, 65, 129)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.25), (errs, rates)


def test_vector_mass_blocks_match_scalar_mass():
    """Each component block of the plain vector mass is the scalar P1 mass."""
    N = 9
    Mv = fem.mass_matrix_vec(N).toarray()
    Ms = fem.mass_matrix(N).toarray()
    assert np.abs(Mv[0::2, 0::2] - Ms).max() < 1e-15
    assert np.abs(Mv[1::2, 1::2] - Ms).max() < 1e-15
    assert np.abs(Mv[0::2, 1::2]).max() == 0.0
