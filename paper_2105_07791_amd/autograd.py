"""Differentiable solve x = A(s)^-1 b through the C ABI.

Forward: factor A(s) (Algorithm 3.4) and run preconditioned GMRES.
Backward (adjoint): for a real loss L with torch's complex gradient
g = dL/dRe(x) + i dL/dIm(x), dL = Re(g^H dx) and dx = -A^-1 (dA) x, so

    mu      = A^-H g                          (GMRES, trans = 2: conj(A^-T conj(g))
                                               with P^-T, conjugations in the library)
    dL/ds_l = -Re( mu^H (dA/ds_l) x )         (hssx_dAds_contract_adjoint)
    dL/db   = mu

All three steps run in libhssx.so; this module only marshals tensors.  A
forward or adjoint solve that stops at its iteration limit raises.
A batch of uneven problems (N and omega given as lists) is one
block-diagonal operator: s, b and x are the parts' vectors stacked.

With a cache (any dict) the factor of a grid configuration is built once and
later calls on the same grids recompute only its numeric factorization
(hssx_refactor), as in an inversion loop that reassembles A(s) every step.
A cached factor is refactored in place: run a call's backward before the
next forward that reuses the cache.
"""
import torch

from .hssx import BatchOperator, Factor, Operator, gmres_solve


def _operator(s, N, omega):
    if isinstance(N, (list, tuple)):
        om = list(omega) if isinstance(omega, (list, tuple)) else [omega] * len(N)
        parts, o = [], 0
        for Nq, wq in zip(N, om):
            parts.append(Operator(int(Nq), float(wq), s[o:o + Nq * Nq]))
            o += Nq * Nq
        assert o == s.numel(), "slowness length does not match the grids"
        return BatchOperator(parts)
    return Operator(N, omega, s)

__all__ = ["WaveSolve", "solve"]


def _require_converged(stats, which):
    """A solve that stopped at maxit leaves x (or the gradient) wrong: fail."""
    bad = [i for i, s in enumerate(stats) if not s["converged"]]
    if bad:
        raise RuntimeError(f"{which} GMRES did not converge for systems {bad[:8]}: "
                           f"{stats[bad[0]]}")


class WaveSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, s, b, N, omega, opts):
        opts = dict(opts or {})
        gm = dict(m=opts.pop("gmres_m", 50), tol=opts.pop("gmres_tol", 1e-8),
                  flexible=opts.pop("flexible", False))
        cache = opts.pop("cache", None)
        A = _operator(s.detach(), N, omega)
        key = (tuple(N) if isinstance(N, (list, tuple)) else N,
               tuple(omega) if isinstance(omega, (list, tuple)) else omega,
               tuple(sorted(opts.items())))
        P = cache.get(key) if cache is not None else None
        if P is None:
            P = Factor(A, **opts)
            if cache is not None:
                cache[key] = P
        else:
            P.refactor(A)
        x, st = gmres_solve(A, P, b.detach(), **gm)
        _require_converged(st, "forward")
        ctx.A, ctx.P, ctx.gm, ctx.stats = A, P, gm, st
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        A, P, gm = ctx.A, ctx.P, ctx.gm
        # adjoint state mu = A^-H dJ/dx (conjugations inside the library)
        mu, st = gmres_solve(A, P, gx, trans="adjoint", **gm)
        _require_converged(st, "adjoint")
        gs = A.dAds_contract(mu, x, adjoint=True) if ctx.needs_input_grad[0] else None
        gb = mu if ctx.needs_input_grad[1] else None
        return gs, gb, None, None, None


def solve(s, b, N, omega, cache=None, **opts):
    """x = A(s)^-1 b, differentiable in the slowness s and the load b.  N and
    omega may be lists (a batch of problems, vectors stacked part by part).
    cache: optional dict for analysis reuse across calls (see module doc)."""
    if cache is not None:
        opts["cache"] = cache
    return WaveSolve.apply(s, b, N, omega, opts)
