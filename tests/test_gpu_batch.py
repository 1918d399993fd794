"""GPU parity of the batching form: uneven problems fused into one forest
factorization and one GMRES with a Krylov basis per (problem, right-hand
side), against the oracle run problem by problem."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import adjoint, approx, exact, fem, nd  # noqa: E402
from synth import make_batch  # noqa: E402


def _hx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2105_07791_amd import hssx
    return hssx


def _batch(bp):
    hx = _hx()
    ops = [hx.Operator(p.N, p.omega, p.slowness) for p in bp.problems]
    return hx.BatchOperator(ops)


def test_forest_matches_per_problem_trees():
    """The batch factor's elimination order is each problem's oracle order,
    shifted by the problem's row offset (bit-exact)."""
    hx = _hx()
    bp = make_batch("helmholtz_p1_batch8")
    A = _batch(bp)
    P = hx.Factor(A, tol=1e-6, h_sw=2)
    perm = P.perm()
    want = np.concatenate([nd.build_nd(p.N, 32, 16).perm + A.part_off[q]
                           for q, p in enumerate(bp.problems)])
    assert np.array_equal(perm, want)


@pytest.mark.parametrize("h_sw", [-1, 2])
def test_batch_apply_matches_oracle(h_sw):
    hx = _hx()
    dev = torch.device("cuda:0")
    bp = make_batch("helmholtz_p1_batch8")
    A = _batch(bp)
    P = hx.Factor(A, tol=1e-6, h_sw=h_sw, seed=3)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((A.n, 2)) + 1j * rng.standard_normal((A.n, 2))
    y = P.apply(torch.tensor(x, device=dev)).cpu().numpy()
    for q, p in enumerate(bp.problems):
        sl = slice(A.part_off[q], A.part_off[q + 1])
        Ao = fem.assemble_helmholtz(p.N, p.omega, p.slowness)
        ye = exact.factor_exact(Ao, nd.build_nd(p.N, 32, 16), keep_S=False).apply(x[sl])
        rel = np.linalg.norm(y[sl] - ye) / np.linalg.norm(ye)
        assert rel <= (1e-11 if h_sw < 0 else 1e-4), (q, p.N, rel)


@pytest.mark.parametrize("dtype,flexible", [("c128", False), ("c64", True)])
def test_batch_gmres_per_problem(dtype, flexible):
    hx = _hx()
    dev = torch.device("cuda:0")
    bp = make_batch("helmholtz_p1_batch8")
    A = _batch(bp)
    P = hx.Factor(A, tol=1e-6, h_sw=2, dtype=dtype)
    f = np.zeros((A.n, 2))
    rng = np.random.default_rng(2)
    for q, p in enumerate(bp.problems):
        f[A.part_off[q]:A.part_off[q + 1], 0] = p.f[:, 0]
        f[A.part_off[q]:A.part_off[q + 1], 1] = rng.standard_normal(p.n)
    b = A.load(torch.tensor(f, device=dev))
    x, st = hx.gmres_solve(A, P, b, flexible=flexible)
    assert len(st) == 2 * A.parts
    xg = x.cpu().numpy()
    for r in range(2):
        for q, p in enumerate(bp.problems):
            s = st[r * A.parts + q]
            assert s["converged"] and s["true_res"] <= 1e-8, (r, q, s)
            sl = slice(A.part_off[q], A.part_off[q + 1])
            Ao = fem.assemble_helmholtz(p.N, p.omega, p.slowness)
            bo = fem.mass_matrix(p.N) @ f[sl, r] + 0j
            xo = exact.factor_exact(Ao, nd.build_nd(p.N, 32, 16), keep_S=False).apply(bo)
            assert np.linalg.norm(Ao @ xg[sl, r] - bo) <= 1e-8 * np.linalg.norm(bo)
            assert np.linalg.norm(xg[sl, r] - xo) <= 1e-6 * np.linalg.norm(xo)


def test_batch_gradient_matches_oracle():
    """Misfit J = sum over problems of 1/2 ||R x - d||^2 and its slowness
    gradient through one batched adjoint solve, against the oracle problem by
    problem."""
    _hx()
    from paper_2105_07791_amd.autograd import solve
    dev = torch.device("cuda:0")
    bp = make_batch("helmholtz_p1_batch8", count=4, lo=9, hi=33)
    Ns = [p.N for p in bp.problems]
    om = [p.omega for p in bp.problems]
    s_all = np.concatenate([p.slowness for p in bp.problems])
    b_all = np.concatenate([fem.mass_matrix(p.N) @ p.f[:, 0] + 0j for p in bp.problems])
    st = torch.tensor(s_all, device=dev, requires_grad=True)
    bt = torch.tensor(b_all, device=dev)
    x = solve(st, bt, Ns, om, h_sw=2, tol=1e-8, gmres_tol=1e-13, dtype="c64", flexible=True)
    J = 0
    off = 0
    for q, p in enumerate(bp.problems):
        rec = torch.tensor(bp.receivers[q] + off, device=dev)
        r = x[rec] - torch.tensor(bp.data[q][:, 0], device=dev)
        J = J + 0.5 * (r.abs() ** 2).sum()
        off += p.n
    J.backward()
    g = st.grad.cpu().numpy()
    off = 0
    Jo_tot = 0.0
    for q, p in enumerate(bp.problems):
        Jo, gso, _, _ = adjoint.misfit_and_gradient(p.N, p.omega, p.slowness,
                                                    b_all[off:off + p.n, None],
                                                    bp.receivers[q], bp.data[q])
        Jo_tot += Jo
        gq = g[off:off + p.n]
        assert np.linalg.norm(gq - gso) <= 1e-6 * np.linalg.norm(gso), q
        off += p.n
    assert abs(J.item() - Jo_tot) <= 1e-9 * Jo_tot


def test_c5_form_split_bf16_uneven_batch():
    """The batch form as the 256-problem workload runs it (split-bf16
    sampling products with fp32 accumulation, complex64 factor, tol 1e-3,
    flexible FP64 GMRES) on 16 problems of 65..513 nodes per side: forward
    misfit against the oracle, slowness gradient against central finite
    differences along seeded directions and, on three of the problems,
    against the oracle's adjoint gradient at sampled nodes."""
    _hx()
    from paper_2105_07791_amd.autograd import solve
    dev = torch.device("cuda:0")
    bp = make_batch("helmholtz_p1_batch16")
    Ns = [p.N for p in bp.problems]
    assert len(Ns) == 16 and min(Ns) < 150 and max(Ns) > 400
    om = [p.omega for p in bp.problems]
    s_all = np.concatenate([p.slowness for p in bp.problems])
    b_all = np.concatenate([fem.mass_matrix(p.N) @ p.f[:, 0] + 0j for p in bp.problems])
    kw = dict(h_sw=4, tol=1e-3, dtype="c64", sample_bf16=2, flexible=True, gmres_tol=1e-12)
    offs = np.cumsum([0] + [p.n for p in bp.problems])

    def J_of(s_vec, grad=False):
        st = torch.tensor(s_vec, device=dev, requires_grad=grad)
        x = solve(st, torch.tensor(b_all, device=dev), Ns, om, **kw)
        J = 0
        for q, p in enumerate(bp.problems):
            rec = torch.tensor(bp.receivers[q] + offs[q], device=dev)
            r = x[rec] - torch.tensor(bp.data[q][:, 0], device=dev)
            J = J + 0.5 * (r.abs() ** 2).sum()
        if grad:
            J.backward()
            return J.item(), st.grad.cpu().numpy(), x.detach().cpu().numpy()
        return J.item()

    J, g, x = J_of(s_all, grad=True)
    # forward: solutions and misfit against direct sparse solves of the
    # oracle's matrices (the plain definition x = A^-1 b; the oracle's own
    # nested dissection of 16 grids up to 500^2 would exceed the test budget)
    import scipy.sparse.linalg as spla
    Jo, lus = 0.0, {}
    for q, p in enumerate(bp.problems):
        Ao = fem.assemble_helmholtz(p.N, p.omega, p.slowness).tocsc()
        lus[q] = (Ao, spla.splu(Ao))
        xo = lus[q][1].solve(b_all[offs[q]:offs[q + 1]])
        assert np.linalg.norm(x[offs[q]:offs[q + 1]] - xo) <= 1e-6 * np.linalg.norm(xo), q
        Jo += 0.5 * float(np.sum(np.abs(xo[bp.receivers[q]] - bp.data[q][:, 0]) ** 2))
    assert abs(J - Jo) <= 1e-8 * Jo
    # gradient: central differences along two seeded directions
    rng = np.random.default_rng(4)
    eps = 1e-4 * np.abs(s_all).max()
    for _ in range(2):
        v = rng.standard_normal(s_all.size)
        fd = (J_of(s_all + eps * v) - J_of(s_all - eps * v)) / (2 * eps)
        assert abs(fd - g @ v) <= 1e-5 * abs(fd), (fd, g @ v)
    # gradient: the oracle's adjoint definition (lambda = A^-T conj(dJ/dx),
    # dJ/ds_l = -Re lambda^T (dA/ds_l) x with the oracle's dA/ds_l) at sampled
    # nodes of the smallest, a middle and the largest problem
    order = np.argsort(Ns)
    for q in (order[0], order[len(order) // 2], order[-1]):
        p = bp.problems[q]
        Ao, lu = lus[q]
        xq = lu.solve(b_all[offs[q]:offs[q + 1]])
        gr = np.zeros_like(xq)
        gr[bp.receivers[q]] = xq[bp.receivers[q]] - bp.data[q][:, 0]
        lam = lu.solve(np.conj(gr), trans="T")
        nodes = np.random.default_rng(int(q)).choice(p.n, size=8, replace=False)
        go = np.array([-np.real(np.sum(lam * (adjoint.dA_ds(p.N, p.omega, p.slowness, l) @ xq)))
                       for l in nodes])
        gq = g[offs[q] + nodes]
        assert np.linalg.norm(gq - go) <= 1e-5 * np.linalg.norm(go), (q, p.N)
