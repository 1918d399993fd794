"""Pins of the oracle GMRES against textbook properties."""
import numpy as np
import scipy.sparse as sp

from oracle import krylov


def test_distinct_eigenvalues_exact_termination():
    """A = diag(1..5) (x) I_20: the minimal polynomial has degree 5, so
    GMRES terminates in exactly 5 steps when b touches every eigenspace."""
    d = np.repeat(np.arange(1.0, 6.0), 20)
    A = sp.diags(d).tocsr()
    b = np.random.default_rng(0).standard_normal(100) + 1j
    r = krylov.gmres(lambda v: A @ v, None, b, m=50, tol=1e-12)
    assert r.iters == 5
    assert r.true_res < 1e-12
    b2 = np.zeros(100, complex)
    b2[:40] = 1.0                          # only eigenvalues 1 and 2
    r2 = krylov.gmres(lambda v: A @ v, None, b2, m=50, tol=1e-12)
    assert r2.iters == 2


def test_restarted_solution_matches_dense():
    rng = np.random.default_rng(3)
    n = 60
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3 + 1j * rng.standard_normal((n, n)) * 0.1
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for side in ("left", "right"):
        P = np.diag(1.0 / np.diag(A))
        r = krylov.gmres(lambda v: A @ v, lambda v: P @ v, b, m=7, tol=1e-11, side=side)
        x = np.linalg.solve(A, b)
        assert np.linalg.norm(r.x - x) / np.linalg.norm(x) < 1e-9
        assert r.iters > 7                  # needed restarts
