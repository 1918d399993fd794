"""Restarted GMRES, left- and right-(flexible) preconditioned (oracle).

The paper solves P^-1 A x = P^-1 b (eq. 1.2) with restarted GMRES and stops on
the preconditioned relative residual ||P^-1(A x - b)|| / ||P^-1 b|| (Sec. 4).
This oracle is the textbook algorithm (Saad, Iterative Methods, Alg. 6.9 and
the flexible variant 9.6): modified Gram-Schmidt Arnoldi, complex Givens
rotations, x0 = 0.

Stopping rule: a cycle ends when its residual estimate reaches tol (relative
to the preconditioned right-hand side for left preconditioning, to b for the
flexible right-preconditioned form) or after m steps.  After convergence of
the estimate the true residual ||b - A x|| / ||b|| is checked; while it is
above tol, up to three more cycles run with the target scaled by the observed
ratio.  Iterations = total Arnoldi steps.
"""
import numpy as np

__all__ = ["gmres", "GmresResult"]


class GmresResult:
    def __init__(self, x, iters, prec_res, true_res, history, converged):
        self.x = x
        self.iters = iters
        self.prec_res = prec_res
        self.true_res = true_res
        self.history = history
        self.converged = converged


def _givens(a, b):
    """c (real), s (complex) with [c s; -conj(s) c] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0
    if a == 0:
        return 0.0, 1.0
    nu = np.hypot(abs(a), abs(b))
    return abs(a) / nu, (a / abs(a)) * np.conj(b) / nu


def gmres(matvec, precond, b, m=50, tol=1e-8, maxit=1000, side="left",
          extra_cycles=3):
    """Solve A x = b.  matvec(v) = A v, precond(v) = P^-1 v (or None)."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.size
    M = precond if precond is not None else (lambda v: v)
    x = np.zeros(n, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0:
        return GmresResult(x, 0, 0.0, 0.0, [], True)
    pb_norm = np.linalg.norm(M(b)) if side == "left" else bnorm
    target = tol
    iters = 0
    history = []
    extra = 0
    prec_rel = np.inf
    while iters < maxit:
        r = b - matvec(x)
        if side == "left":
            r = M(r)
        beta = np.linalg.norm(r)
        prec_rel = beta / pb_norm
        if prec_rel <= target:
            true_rel = np.linalg.norm(b - matvec(x)) / bnorm
            if true_rel <= tol or extra >= extra_cycles:
                return GmresResult(x, iters, prec_rel, true_rel, history, true_rel <= tol)
            target = target * tol / true_rel
            extra += 1
            continue
        V = np.zeros((n, m + 1), dtype=np.complex128)
        Z = np.zeros((n, m), dtype=np.complex128) if side == "right" else None
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[:, 0] = r / beta
        j_done = 0
        for j in range(m):
            if side == "left":
                w = M(matvec(V[:, j]))
            else:
                Z[:, j] = M(V[:, j])
                w = matvec(Z[:, j])
            for i in range(j + 1):                         # modified Gram-Schmidt
                H[i, j] = np.vdot(V[:, i], w)
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):                              # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            j_done = j + 1
            res = abs(g[j + 1]) / pb_norm
            history.append(res)
            if res <= target or iters >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        if side == "left":
            x = x + V[:, :j_done] @ y
        else:
            x = x + Z[:, :j_done] @ y
    true_rel = np.linalg.norm(b - matvec(x)) / bnorm
    return GmresResult(x, iters, prec_rel, true_rel, history, False)
