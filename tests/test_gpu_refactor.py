"""Numeric refactorization (hssx_refactor): the analysis, descriptors, pools
and apply graphs of a factor are kept while every value is recomputed from a
new operator with the same pattern.  The refactored preconditioner must equal
a fresh factorization of the new operator bit for bit (same sketches, same
kernels), and GMRES with it must solve the new system to the oracle's
residual bar."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import fem  # noqa: E402
from synth import make_dg, make_elastic, make_problem, speed_field  # noqa: E402


def _hx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2105_07791_amd import hssx
    return hssx


@pytest.mark.parametrize("dtype,graph", [("c128", False), ("c64", True)])
def test_refactor_equals_fresh_factor(dtype, graph):
    hx = _hx()
    dev = torch.device("cuda:0")
    pr = make_problem("helmholtz_p1_129")
    s1 = 1.0 / speed_field(pr.N, 11)
    s2 = 1.0 / speed_field(pr.N, 12)
    A1 = hx.Operator(pr.N, pr.omega, s1)
    A2 = hx.Operator(pr.N, pr.omega, s2)
    P = hx.Factor(A1, tol=1e-6, h_sw=3, dtype=dtype, seed=4, apply_graph=graph)
    b = A2.load(torch.tensor(pr.f, device=dev))
    y1 = P.apply(b).clone()          # captures the graphs on the first factor
    P.refactor(A2)
    y2 = P.apply(b)
    Q = hx.Factor(A2, tol=1e-6, h_sw=3, dtype=dtype, seed=4, apply_graph=False)
    yq = Q.apply(b)
    assert torch.equal(y2, yq)
    assert not torch.equal(y1, y2)
    assert P.stats()["k_max"] == Q.stats()["k_max"]
    x, st = hx.gmres_solve(A2, P, b, flexible=dtype == "c64")
    Ao = fem.assemble_helmholtz(pr.N, pr.omega, s2)
    xo, bo = x.cpu().numpy(), b.cpu().numpy()
    for r in range(bo.shape[1]):
        assert st[r]["converged"]
        assert np.linalg.norm(Ao @ xo[:, r] - bo[:, r]) <= 1e-8 * np.linalg.norm(bo[:, r])
    # refactoring the same operator again reproduces the factor exactly
    P.refactor()
    assert torch.equal(P.apply(b), yq)


def test_refactor_other_operators_and_batches():
    hx = _hx()
    dev = torch.device("cuda:0")
    pd = make_dg("sipg_p2_16")
    D1 = hx.DGOperator(pd.Nc, pd.omega, pd.slowness)
    D2 = hx.DGOperator(pd.Nc, pd.omega, 1.1 * pd.slowness)
    P = hx.Factor(D1, tol=1e-6, leaf_size=60, beta=60, h_sw=2, seed=2)
    b = D2.load(torch.tensor(pd.f, device=dev))
    P.refactor(D2)
    Q = hx.Factor(D2, tol=1e-6, leaf_size=60, beta=60, h_sw=2, seed=2)
    assert torch.equal(P.apply(b), Q.apply(b))
    pe = make_elastic("elastic_p1_33")
    E1 = hx.ElasticOperator(pe.N, pe.omega, pe.lam, pe.mu, pe.rho)
    E2 = hx.ElasticOperator(pe.N, pe.omega, pe.lam, 1.2 * pe.mu, pe.rho)
    P = hx.Factor(E1, tol=1e-6, leaf_size=64, beta=32, h_sw=2, seed=2)
    b = E2.load(torch.tensor(pe.f, device=dev))
    P.refactor(E2)
    Q = hx.Factor(E2, tol=1e-6, leaf_size=64, beta=32, h_sw=2, seed=2)
    assert torch.equal(P.apply(b), Q.apply(b))
    # batches of the same grids
    Ns = [17, 33, 25]
    mk = lambda seed: hx.BatchOperator([hx.Operator(N, 0.25 * (N - 1),  # noqa: E731
                                                    1.0 / speed_field(N, seed + N)) for N in Ns])
    B1, B2 = mk(1), mk(2)
    P = hx.Factor(B1, tol=1e-6, h_sw=2, dtype="c64", seed=3)
    x = torch.randn(B2.n, 2, dtype=torch.complex128, device=dev)
    P.refactor(B2)
    Q = hx.Factor(B2, tol=1e-6, h_sw=2, dtype="c64", seed=3)
    assert torch.equal(P.apply(x), Q.apply(x))


def test_refactor_rejects_other_patterns():
    hx = _hx()
    from paper_2105_07791_amd._lib import HssxError
    pr = make_problem("helmholtz_p1_17")
    A = hx.Operator(pr.N, pr.omega, pr.slowness)
    P = hx.Factor(A, tol=1e-6)
    with pytest.raises(HssxError):
        P.refactor(hx.Operator(pr.N + 1, pr.omega, np.ones((pr.N + 1) ** 2)))
    pe = make_elastic("elastic_p1_33", N=pr.N)
    with pytest.raises(HssxError):
        P.refactor(hx.ElasticOperator(pe.N, pe.omega, pe.lam, pe.mu, pe.rho))
    # still usable with its own operator
    P.refactor(A)


def test_autograd_cache_matches_fresh_factors():
    """An inversion-style loop with a factor cache gives the same solutions
    and slowness gradients as fresh factorizations, step after step."""
    _hx()
    from paper_2105_07791_amd.autograd import solve
    dev = torch.device("cuda:0")
    Ns = [17, 29]
    om = [0.25 * (N - 1) for N in Ns]
    f = torch.randn(sum(N * N for N in Ns), dtype=torch.float64, device=dev)
    from paper_2105_07791_amd.hssx import BatchOperator, Operator
    b = BatchOperator([Operator(N, w, np.ones(N * N)) for N, w in zip(Ns, om)]).load(f)
    opts = dict(tol=1e-6, h_sw=2, dtype="c64", flexible=True, seed=1)
    cache = {}
    for seed in (1, 2, 3):
        s = torch.cat([1.0 / speed_field(N, seed + N, device=dev) for N in Ns])
        grads, xs = [], []
        for c in (cache, None):
            st = s.clone().requires_grad_(True)
            x = solve(st, b, Ns, om, cache=c, **opts)
            (0.5 * (x.abs() ** 2).sum()).backward()
            grads.append(st.grad)
            xs.append(x.detach())
        assert torch.equal(xs[0], xs[1])
        assert torch.equal(grads[0], grads[1])
    assert len(cache) == 1
