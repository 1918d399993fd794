"""Pins of the oracle's approximate factorization (Algorithm 3.4): it is an
exact solver in the limit of vanishing tolerance, a good preconditioner at the
working tolerance, and its compressions meet their tolerance."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import approx, exact, fem, krylov, nd
from synth import make_problem


def _setup(N, om, leaf=32, beta=16):
    A = fem.assemble_helmholtz(N, om)
    t = nd.build_nd(N, leaf, beta)
    pr = make_problem("helmholtz_p1_65", N=N, omega=om)
    b = (fem.mass_matrix(N) @ pr.f[:, 0]).astype(complex)
    return A, t, b


def test_vanishing_tolerance_is_exact():
    A, t, b = _setup(33, 8.0)
    fe = exact.factor_exact(A, t)
    fa = approx.factor_approx(A, t, h_sw=2, tol=1e-14, id_rel_tol=1e-15)
    assert sum(a == "hss" for a in fa.arith) > 3
    x = fa.apply(b)
    xe = fe.apply(b)
    assert np.linalg.norm(x - xe) / np.linalg.norm(xe) < 1e-9


@pytest.mark.parametrize("N,om,h_sw", [(33, 8.0, 2), (65, 16.0, 4)])
def test_preconditioned_gmres(N, om, h_sw):
    A, t, b = _setup(N, om)
    fa = approx.factor_approx(A, t, h_sw=h_sw, tol=1e-6, seed=7)
    r = krylov.gmres(lambda v: A @ v, fa.apply, b, m=50, tol=1e-8)
    xr = spla.spsolve(A.tocsc(), b)
    assert r.iters <= 5
    assert r.true_res <= 1e-8
    assert np.linalg.norm(r.x - xr) / np.linalg.norm(xr) <= 1e-6
    for k, H in fa.S_hss.items():
        assert H.est <= 1e-6
    for k in fa.R:
        assert np.array_equal(fa.L[k], fa.R[k].T)


def test_transpose_apply_equals_apply():
    A, t, b = _setup(33, 8.0)
    fa = approx.factor_approx(A, t, h_sw=2, tol=1e-6)
    y1 = fa.apply(b)
    y2 = fa.apply_t(b)
    assert np.linalg.norm(y1 - y2) / np.linalg.norm(y1) < 1e-8
