"""Pins of the oracle's exact elimination (eqs. 3.2-3.5, Algorithm 3.1)
against brute-force dense linear algebra."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import exact, fem, krylov, nd


@pytest.mark.parametrize("N,om,leaf", [(9, 3.0, 8), (17, 4.0, 32), (33, 8.0, 32), (20, 5.0, 12)])
def test_solve_matches_dense(N, om, leaf):
    A = fem.assemble_helmholtz(N, om, np.linspace(0.8, 1.2, N * N))
    t = nd.build_nd(N, leaf, 8)
    f = exact.factor_exact(A, t)
    rng = np.random.default_rng(N)
    b = rng.standard_normal((N * N, 2)) + 1j * rng.standard_normal((N * N, 2))
    x = f.apply(b)
    xr = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) < 1e-12
    xt = f.apply_t(b)                   # A^T = A, so P^-T = P^-1 exactly
    assert np.linalg.norm(xt - xr) / np.linalg.norm(xr) < 1e-12


def test_schur_complements_are_box_schur():
    """S(sigma) = A_BB - A_BI A_II^-1 A_IB for the box submatrix of sigma,
    B = Bd(sigma), I = box minus Bd(sigma): the definition of eq. 3.5 unrolled
    over the subtree."""
    N = 17
    A = fem.assemble_helmholtz(N, 4.0)
    t = nd.build_nd(N, 16, 8)
    f = exact.factor_exact(A, t)
    Ad = A.toarray()
    for k, b in enumerate(t.boxes[:-1]):
        xs = np.arange(b.x0, b.x1)
        ys = np.arange(b.y0, b.y1)
        box = (ys[:, None] * N + xs[None, :]).ravel()
        Bset = b.B
        Iset = np.setdiff1d(box, Bset)
        S = Ad[np.ix_(Bset, Bset)] - Ad[np.ix_(Bset, Iset)] @ np.linalg.solve(
            Ad[np.ix_(Iset, Iset)], Ad[np.ix_(Iset, Bset)])
        assert np.linalg.norm(f.S[k] - S) <= 1e-12 * np.linalg.norm(S)


def test_ldr_reconstruction_and_symmetry():
    N = 9
    A = fem.assemble_helmholtz(N, 3.0)
    t = nd.build_nd(N, 8, 4)
    f = exact.factor_exact(A, t)
    Pinv = f.apply(np.eye(N * N))
    Ad = A.toarray()
    assert np.linalg.norm(Ad @ Pinv - np.eye(N * N)) < 1e-12 * N * N
    for k in f.R:
        assert np.linalg.norm(f.L[k] - f.R[k].T) <= 1e-12 * np.linalg.norm(f.R[k])


def test_gmres_one_iteration_with_exact_factor():
    N = 33
    A = fem.assemble_helmholtz(N, 8.0)
    t = nd.build_nd(N)
    f = exact.factor_exact(A, t)
    b = np.random.default_rng(1).standard_normal(N * N) + 0j
    r = krylov.gmres(lambda v: A @ v, f.apply, b, m=50, tol=1e-8)
    assert r.iters == 1
    assert r.prec_res < 1e-12 and r.true_res < 1e-12
