"""Pin of the oracle adjoint gradient (dJ/ds, dJ/db of J = 1/2 ||x[rec] - d||^2,
x = A(s)^-1 b) against central finite differences of J, computed with the
oracle's exact solver."""
import numpy as np

from oracle import adjoint, exact, fem, nd


def _J(N, om, s, b, rec, d):
    A = fem.assemble_helmholtz(N, om, s)
    f = exact.factor_exact(A, nd.build_nd(N, 32, 16), keep_S=False)
    x = f.apply(b)
    return 0.5 * float(np.sum(np.abs(x[rec] - d) ** 2))


def test_gradient_matches_central_differences():
    N, om = 9, 3.0
    rng = np.random.default_rng(0)
    s = 1.0 + 0.2 * rng.random(N * N)
    b = rng.standard_normal((N * N, 2)) + 1j * rng.standard_normal((N * N, 2))
    rec = np.array([3, 17, 40, 77])
    d = rng.standard_normal((4, 2)) + 1j * rng.standard_normal((4, 2))
    J, gs, gb, x = adjoint.misfit_and_gradient(N, om, s, b, rec, d)
    assert abs(J - _J(N, om, s, b, rec, d)) < 1e-12 * J
    for k in range(3):
        v = rng.standard_normal(N * N)
        eps = 1e-5
        fd = (_J(N, om, s + eps * v, b, rec, d) - _J(N, om, s - eps * v, b, rec, d)) / (2 * eps)
        assert abs(fd - gs @ v) <= 1e-6 * abs(fd)
    # db: dJ = Re(gb^H db)
    db = rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape)
    eps = 1e-6
    fd = (_J(N, om, s, b + eps * db, rec, d) - _J(N, om, s, b - eps * db, rec, d)) / (2 * eps)
    assert abs(fd - np.real(np.vdot(gb, db))) <= 1e-6 * abs(fd)


def test_dA_ds_sums_to_dA_dscale():
    """sum_l s_l dA/ds_l = d/dt A(t s) at t = 1 = -2 omega^2 M[s^2] - i omega G[s]
    (the weights are homogeneous of degree 2 and 1)."""
    N, om = 6, 2.0
    s = np.linspace(0.7, 1.3, N * N)
    tot = sum(s[l] * adjoint.dA_ds(N, om, s, l) for l in range(N * N))
    A1 = fem.assemble_helmholtz(N, om, s)
    h = 1e-6
    Ap = fem.assemble_helmholtz(N, om, s * (1 + h))
    Am = fem.assemble_helmholtz(N, om, s * (1 - h))
    fd = (Ap - Am) / (2 * h)
    assert abs(tot - fd).max() <= 1e-7 * abs(A1).max()
