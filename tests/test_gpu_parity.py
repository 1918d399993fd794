"""GPU parity: the HIP path (through the C ABI) against the oracle on the same
seeded inputs.  Bars: integer/index work bit-exact (covered on the CPU by
test_abi_cpu); FP64 assembly and exact elimination to rounding (1e-12
relative); the compressed preconditioner to its tolerance; GMRES solutions
to a true relative residual of 1e-8 and a solution error of 1e-6 against the
oracle's exact solve."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import approx, exact, fem, nd  # noqa: E402
from synth import make_problem, speed_field  # noqa: E402


def _dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def _hssx():
    from paper_2105_07791_amd import hssx
    return hssx


def _problem(N, om, nsrc=2, seed=3, variable=False):
    pr = make_problem("helmholtz_p1_65", N=N, omega=om, seed=seed, nsrc=nsrc)
    s = 1.0 / speed_field(N, seed) if variable else np.ones(N * N)
    return pr, s


@pytest.mark.parametrize("N,om,variable", [(9, 3.0, False), (65, 16.0, True), (130, 20.0, True)])
def test_assembly_load_spmv(N, om, variable):
    dev = _dev()
    hx = _hssx()
    pr, s = _problem(N, om, variable=variable)
    A = hx.Operator(N, om, s)
    rp, col, val = A.csr()
    Ao = fem.assemble_helmholtz(N, om, s)
    assert np.array_equal(rp, Ao.indptr) and np.array_equal(col, Ao.indices)
    assert np.abs(val - Ao.data).max() <= 1e-13 * np.abs(Ao.data).max()
    # bitwise symmetry of the device assembly
    import scipy.sparse as sp
    Ag = sp.csr_matrix((val, col, rp), shape=Ao.shape)
    assert (Ag != Ag.T).nnz == 0
    f = torch.tensor(pr.f, device=dev)
    b = A.load(f).cpu().numpy()
    bo = fem.mass_matrix(N) @ pr.f
    assert np.abs(b - bo).max() <= 1e-14 * np.abs(bo).max()
    x = np.random.default_rng(0).standard_normal((N * N, 3)) + 1j
    y = A.matvec(torch.tensor(x, device=dev)).cpu().numpy()
    yo = Ao @ x
    assert np.linalg.norm(y - yo) <= 1e-13 * np.linalg.norm(yo)


@pytest.mark.parametrize("N,om,leaf", [(17, 4.0, 32), (40, 9.0, 20), (65, 16.0, 32)])
def test_exact_factor(N, om, leaf):
    """h_sw < 0: no compression, the factor is the exact sparse direct solver."""
    dev = _dev()
    hx = _hssx()
    pr, s = _problem(N, om)
    A = hx.Operator(N, om, s)
    P = hx.Factor(A, tol=1e-6, leaf_size=leaf, h_sw=-1)
    Ao = fem.assemble_helmholtz(N, om, s)
    t = nd.build_nd(N, leaf, 16)
    fo = exact.factor_exact(Ao, t)
    b = fem.mass_matrix(N) @ pr.f + 0j
    y = P.apply(torch.tensor(b, device=dev)).cpu().numpy()
    yo = fo.apply(b)
    assert np.linalg.norm(y - yo) <= 1e-11 * np.linalg.norm(yo)
    yt = P.apply(torch.tensor(b, device=dev), trans=True).cpu().numpy()
    assert np.linalg.norm(yt - yo) <= 1e-11 * np.linalg.norm(yo)
    for k in range(0, len(t.boxes) - 1, max(1, len(t.boxes) // 7)):
        S = P.schur(k, t.boxes[k].B.size)
        assert np.linalg.norm(S - fo.S[k]) <= 1e-11 * np.linalg.norm(fo.S[k])
    x, st = hx.gmres_solve(A, P, torch.tensor(b, device=dev))
    assert all(v["iters"] == 1 for v in st)
    assert all(v["true_res"] < 1e-12 for v in st)


@pytest.mark.parametrize("N,om,h_sw", [(33, 8.0, 2), (65, 16.0, 4)])
def test_compressed_factor_matches_oracle(N, om, h_sw):
    dev = _dev()
    hx = _hssx()
    pr, s = _problem(N, om)
    A = hx.Operator(N, om, s)
    P = hx.Factor(A, tol=1e-6, leaf_size=32, beta=16, h_sw=h_sw, seed=5)
    st = P.stats()
    assert st["n_hss_nodes"] > 0 and st["n_compressed"] > 0
    assert st["max_estimate"] <= 1e-6
    Ao = fem.assemble_helmholtz(N, om, s)
    t = nd.build_nd(N, 32, 16)
    fa = approx.factor_approx(Ao, t, h_sw=h_sw, tol=1e-6, seed=5)
    fe = exact.factor_exact(Ao, t, keep_S=False)
    b = fem.mass_matrix(N) @ pr.f + 0j
    y = P.apply(torch.tensor(b, device=dev)).cpu().numpy()
    ya = fa.apply(b)
    ye = fe.apply(b)
    # both are preconditioners within the compression tolerance of A^-1
    assert np.linalg.norm(y - ya) <= 1e-5 * np.linalg.norm(ye)
    assert np.linalg.norm(y - ye) <= 1e-4 * np.linalg.norm(ye)
    x, stats = hx.gmres_solve(A, P, torch.tensor(b, device=dev), m=50, tol=1e-8)
    x = x.cpu().numpy()
    for r in range(b.shape[1]):
        assert stats[r]["converged"] and stats[r]["true_res"] <= 1e-8
        assert stats[r]["iters"] <= 6
        assert np.linalg.norm(x[:, r] - ye[:, r]) <= 1e-6 * np.linalg.norm(ye[:, r])
        assert np.linalg.norm(Ao @ x[:, r] - b[:, r]) <= 1e-8 * np.linalg.norm(b[:, r])


def test_mixed_precision_flexible():
    """c64 factor inside FP64 flexible GMRES reaches the FP64 target."""
    dev = _dev()
    hx = _hssx()
    N, om = 65, 16.0
    pr, s = _problem(N, om, nsrc=4)
    A = hx.Operator(N, om, s)
    P = hx.Factor(A, tol=1e-4, h_sw=4, dtype="c64", seed=1)
    b = A.load(torch.tensor(pr.f, device=dev))
    x, stats = hx.gmres_solve(A, P, b, flexible=True)
    Ao = fem.assemble_helmholtz(N, om, s)
    bo = b.cpu().numpy()
    xo = x.cpu().numpy()
    import scipy.sparse.linalg as spla
    xe = spla.splu(Ao.tocsc()).solve(bo)
    for r in range(bo.shape[1]):
        assert stats[r]["converged"]
        assert np.linalg.norm(Ao @ xo[:, r] - bo[:, r]) <= 1e-8 * np.linalg.norm(bo[:, r])
        assert np.linalg.norm(xo[:, r] - xe[:, r]) <= 1e-6 * np.linalg.norm(xe[:, r])


def test_batched_rhs_equal_single():
    dev = _dev()
    hx = _hssx()
    N, om = 33, 8.0
    pr, s = _problem(N, om, nsrc=5)
    A = hx.Operator(N, om, s)
    P = hx.Factor(A, tol=1e-6, h_sw=2)
    b = A.load(torch.tensor(pr.f, device=dev))
    y = P.apply(b).cpu().numpy()
    for r in range(5):
        yr = P.apply(b[:, r].contiguous()).cpu().numpy()
        assert np.array_equal(yr, y[:, r])
    xb, _ = hx.gmres_solve(A, P, b)
    x2, _ = hx.gmres_solve(A, P, b[:, 2].contiguous())
    assert np.linalg.norm(xb[:, 2].cpu().numpy() - x2.cpu().numpy()) <= 1e-12 * np.linalg.norm(
        x2.cpu().numpy())


def test_errors_are_reported():
    _dev()
    hx = _hssx()
    from paper_2105_07791_amd._lib import HssxError
    A = hx.Operator(9, 2.0, np.ones(81))
    with pytest.raises(HssxError):
        hx.Factor(A, tol=0.0)
    with pytest.raises(HssxError):
        hx.Factor(A, tol=1e-6, leaf_size=0)


def test_compression_stopped_above_tol_is_reported():
    """A compression that stops at its round limit above tol is counted in the
    factor statistics, and fails the factorization in strict mode."""
    _dev()
    hx = _hssx()
    from paper_2105_07791_amd._lib import HSSX_ERANKCAP, HssxError
    N, om = 33, 8.0
    A = hx.Operator(N, om, np.ones(N * N))
    kw = dict(tol=1e-12, leaf_size=32, beta=16, h_sw=1, k0=2, r=2, max_rounds=1)
    P = hx.Factor(A, **kw)
    st = P.stats()
    assert st["n_above_tol"] > 0 and st["max_estimate"] > 1e-12
    with pytest.raises(HssxError) as e:
        hx.Factor(A, strict_tol=True, **kw)
    assert e.value.code == HSSX_ERANKCAP
    P2 = hx.Factor(A, tol=1e-6, leaf_size=32, beta=16, h_sw=1, strict_tol=True)
    assert P2.stats()["n_above_tol"] == 0
