"""Adjoint gradient of a real functional through x = A(s)^-1 b (oracle).

With g = dL/dRe(x) + i dL/dIm(x) (so dL = Re(g^H dx)) and dx = -A^-1 dA x:

    lambda   = A^-T conj(g)
    dL/ds_l  = -Re( lambda^T (dA/ds_l) x )
    dL/db    = conj(lambda)

A(s) = K - omega^2 M[s^2] - i omega G[s] is linear in the nodal weights of
M and G, so dA/ds_l = -2 omega^2 s_l M[e_l] - i omega G[e_l], assembled here
with the oracle's own element routine for each unit nodal vector e_l
(plain and slow, small grids only).  Solves use the exact multifrontal
factor.
"""
import numpy as np

from . import exact, fem, nd

__all__ = ["misfit_and_gradient", "dA_ds"]


def dA_ds(N, omega, s, l):
    """Sparse dA/ds_l."""
    e = np.zeros(N * N)
    e[l] = 1.0
    rows, cols, v = fem.assemble_parts(N, e)      # M[e_l^2] = M[e_l], G[e_l]
    val = -2.0 * omega * omega * s[l] * v["M2"] - 1j * omega * v["G"]
    return fem._mirror_csr(N * N, rows, cols, val.astype(np.complex128))


def misfit_and_gradient(N, omega, s, b, rec, d, leaf=32, beta=16):
    """J = 1/2 sum_r ||x_r[rec] - d_r||^2 and dJ/ds, dJ/db for x = A(s)^-1 b."""
    A = fem.assemble_helmholtz(N, omega, s)
    t = nd.build_nd(N, leaf, beta)
    f = exact.factor_exact(A, t, keep_S=False)
    x = f.apply(b)
    res = x[rec] - d
    J = 0.5 * float(np.sum(np.abs(res) ** 2))
    g = np.zeros_like(x)
    g[rec] = res                                   # dJ/dRe x + i dJ/dIm x
    lam = f.apply_t(np.conj(g))                    # A^-T conj(g)
    grad = np.empty(N * N)
    for l in range(N * N):
        grad[l] = -np.real(np.sum(lam * (dA_ds(N, omega, s, l) @ x)))
    return J, grad, np.conj(lam), x
