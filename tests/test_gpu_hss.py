"""GPU parity of the HSS arithmetic (Sec. 2.2, Sec. 3.3-3.5) through the C ABI.

Kernel level (hssx_hss_eval on oracle-generated HSS matrices, against the
oracle's dense expansion H.dense()):
  * the telescoping product H X;
  * the telescoping inverse H^-1 X against a dense solve with the expansion;
  * entry access H(i, j) and H^-1(i, j).
Factor level (the matrix-free factorization of the HSS-class nodes):
  * GMRES solutions against the oracle's exact nested-dissection solve;
  * with a tiny tolerance the preconditioner approaches A^-1;
  * compressed Schur complements against the oracle's exact ones;
  * the factorization's nominal flops and apply bytes below the exact
    multifrontal factorization of the same tree.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import exact, fem, hss, nd  # noqa: E402
from synth import make_problem  # noqa: E402


def _dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def _hssx():
    from paper_2105_07791_amd import hssx
    return hssx


def _pack(H):
    """Oracle HSS -> (tree rows, ranks, packed generators) of hssx_hss_eval."""
    t = H.tree
    ncl = t.nclusters
    tree = np.stack([t.start, t.size, t.left, t.right, t.level], 1).astype(np.int32)
    rank = np.array([0 if c == 0 else H.U[c].shape[1] for c in range(ncl)], dtype=np.int32)
    parts = []
    for c in range(ncl):
        if c > 0:
            parts.append(H.U[c].ravel(order="F"))
        if t.left[c] < 0:
            parts.append(H.D[c].ravel(order="F"))
        else:
            parts += [H.B12[c].ravel(order="F"), H.B21[c].ravel(order="F")]
    return tree, rank, np.concatenate(parts).astype(np.complex128)


def _trees():
    t65 = nd.build_nd(65, 32, 16)
    t129 = nd.build_nd(129, 32, 16)
    return {
        "c1_root_child": t65.boxes[t65.boxes[-1].lo].ctree,     # [P0 | P1] split
        "c129_root_child": t129.boxes[t129.boxes[-1].lo].ctree,
        "c129_mid": t129.boxes[t129.boxes[-1].lo - 3].ctree,
    }


def _random(ct, k, seed, shift):
    """random_hss with its leaf blocks shifted by shift * I (conditioning)."""
    H = hss.random_hss(ct, k, seed=seed)
    for c in H.D:
        H.D[c] = H.D[c] + shift * np.eye(H.D[c].shape[0])
    return H


@pytest.mark.parametrize("name", ["c1_root_child", "c129_root_child", "c129_mid"])
@pytest.mark.parametrize("dtype,tol", [("c128", 1e-12), ("c64", 2e-5)])
def test_telescoping_product(name, dtype, tol):
    dev = _dev()
    hx = _hssx()
    ct = _trees()[name]
    H = _random(ct, 6, seed=3, shift=4.0)
    Hd = H.dense()
    X = np.random.default_rng(1).standard_normal((Hd.shape[0], 5)) * (1 + 0.5j)
    Y = hx.hss_eval(*_pack(H), 0, X=torch.tensor(X, device=dev), dtype=dtype).cpu().numpy()
    assert np.linalg.norm(Y - Hd @ X) <= tol * np.linalg.norm(Hd @ X)


@pytest.mark.parametrize("name", ["c1_root_child", "c129_root_child", "c129_mid"])
@pytest.mark.parametrize("dtype,tol", [("c128", 1e-10), ("c64", 1e-3)])
def test_telescoping_inverse(name, dtype, tol):
    dev = _dev()
    hx = _hssx()
    ct = _trees()[name]
    H = _random(ct, 6, seed=4, shift=40.0)
    Hd = H.dense()
    assert np.linalg.cond(Hd) < 1e4
    X = np.random.default_rng(2).standard_normal((Hd.shape[0], 3)) + 0.25j
    Y = hx.hss_eval(*_pack(H), 1, X=torch.tensor(X, device=dev), dtype=dtype).cpu().numpy()
    Z = np.linalg.solve(Hd, X)
    assert np.linalg.norm(Y - Z) <= tol * np.linalg.norm(Z)
    assert np.linalg.norm(Hd @ Y - X) <= 10 * tol * np.linalg.norm(X)


@pytest.mark.parametrize("name", ["c1_root_child", "c129_root_child", "c129_mid"])
def test_wide_telescoping_inverse(name):
    """Ops 4 and 5: the complex64 telescoping inverse computed in complex128
    (the factor option wide_inverse) against dense numpy solves and inverses,
    to the bounds of the complex64 ops 1 and 3 on the same matrix."""
    dev = _dev()
    hx = _hssx()
    ct = _trees()[name]
    H = _random(ct, 6, seed=4, shift=40.0)
    Hd = H.dense()
    X = np.random.default_rng(2).standard_normal((Hd.shape[0], 3)) + 0.25j
    Z = np.linalg.solve(Hd, X)
    Xt = torch.tensor(X, device=dev)
    Y4 = hx.hss_eval(*_pack(H), 4, X=Xt, dtype="c64").cpu().numpy()
    assert np.linalg.norm(Y4 - Z) <= 1e-3 * np.linalg.norm(Z)
    assert np.linalg.norm(Hd @ Y4 - X) <= 1e-2 * np.linalg.norm(X)
    m = Hd.shape[0]
    rng = np.random.default_rng(3)
    ij = np.concatenate([rng.integers(0, m, (300, 2)), np.stack([np.arange(m), np.arange(m)], 1)])
    Hi = np.linalg.inv(Hd)[ij[:, 0], ij[:, 1]]
    v5 = hx.hss_eval(*_pack(H), 5, ij=ij, dtype="c64")
    v3 = hx.hss_eval(*_pack(H), 3, ij=ij, dtype="c64")
    scale = np.abs(np.linalg.inv(Hd)).max()
    assert np.abs(v5 - Hi).max() <= 1e-4 * scale
    assert np.abs(v3 - Hi).max() <= 1e-4 * scale
    # complex128: ops 4 and 5 are ops 1 and 3
    Y1 = hx.hss_eval(*_pack(H), 1, X=Xt).cpu().numpy()
    Y4d = hx.hss_eval(*_pack(H), 4, X=Xt).cpu().numpy()
    assert np.array_equal(Y1, Y4d)


@pytest.mark.parametrize("dtype,op", [("c128", 1), ("c64", 1), ("c64", 4)])
def test_singular_leaf_block_reported(dtype, op):
    """A zero leaf block makes the telescoping inverse fail with ESINGULAR
    (the elimination reports its zero pivot); the next call on a regular
    matrix still succeeds."""
    dev = _dev()
    hx = _hssx()
    from paper_2105_07791_amd._lib import HssxError
    ct = _trees()["c129_mid"]
    H = _random(ct, 6, seed=4, shift=40.0)
    X = torch.tensor(np.ones((H.dense().shape[0], 2)) + 0j, device=dev)
    leaf = next(iter(H.D))
    Hz = _random(ct, 6, seed=4, shift=40.0)
    Hz.D[leaf] = np.zeros_like(Hz.D[leaf])
    with pytest.raises(HssxError, match="zero pivot"):
        hx.hss_eval(*_pack(Hz), op, X=X, dtype=dtype)
    Y = hx.hss_eval(*_pack(H), op, X=X, dtype=dtype).cpu().numpy()
    Hd = H.dense()
    Z = np.linalg.solve(Hd, X.cpu().numpy())
    assert np.linalg.norm(Y - Z) <= 1e-3 * np.linalg.norm(Z)


@pytest.mark.parametrize("name", ["c1_root_child", "c129_mid"])
def test_entry_access(name):
    _dev()
    hx = _hssx()
    ct = _trees()[name]
    H = _random(ct, 7, seed=5, shift=40.0)
    Hd = H.dense()
    m = Hd.shape[0]
    rng = np.random.default_rng(3)
    ij = np.concatenate([rng.integers(0, m, (400, 2)),                    # anywhere
                         np.stack([np.arange(m), np.arange(m)], 1),       # diagonal
                         np.stack([np.arange(m - 1), np.arange(1, m)], 1)])  # neighbours
    v = hx.hss_eval(*_pack(H), 2, ij=ij)
    ref = Hd[ij[:, 0], ij[:, 1]]
    assert np.abs(v - ref).max() <= 1e-12 * np.abs(Hd).max()
    vi = hx.hss_eval(*_pack(H), 3, ij=ij)
    Hi = np.linalg.inv(Hd)
    assert np.abs(vi - Hi[ij[:, 0], ij[:, 1]]).max() <= 1e-10 * np.abs(Hi).max()


def test_single_leaf_and_rank_zero():
    """Edge cases: a tree that is one leaf; clusters of rank 0."""
    dev = _dev()
    hx = _hssx()
    rng = np.random.default_rng(7)
    m = 12
    D = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    D = D + D.T + 20 * np.eye(m)
    tree = np.array([[0, m, -1, -1, 0]], dtype=np.int32)
    X = rng.standard_normal((m, 2)) + 0j
    Xd = torch.tensor(X, device=dev)
    Y = hx.hss_eval(tree, [0], D.ravel(order="F"), 0, X=Xd).cpu().numpy()
    assert np.linalg.norm(Y - D @ X) <= 1e-13 * np.linalg.norm(D @ X)
    Y = hx.hss_eval(tree, [0], D.ravel(order="F"), 1, X=Xd).cpu().numpy()
    assert np.linalg.norm(Y - np.linalg.solve(D, X)) <= 1e-12 * np.linalg.norm(np.linalg.solve(D, X))
    ct = _trees()["c1_root_child"]
    H = _random(ct, 0, seed=1, shift=30.0)          # block diagonal: every rank 0
    Hd = H.dense()
    X = rng.standard_normal((Hd.shape[0], 2)) + 0j
    Y = hx.hss_eval(*_pack(H), 1, X=torch.tensor(X, device=dev)).cpu().numpy()
    assert np.linalg.norm(Y - np.linalg.solve(Hd, X)) <= 1e-11 * np.linalg.norm(X)


# ---------------------------------------------------------------- factor level

def _solve_case(N, om, h_sw, tol, dtype, nsrc=3, seed=3):
    dev = _dev()
    hx = _hssx()
    pr = make_problem("helmholtz_p1_65", N=N, omega=om, seed=seed, nsrc=nsrc)
    s = np.ones(N * N)
    A = hx.Operator(N, om, s)
    P = hx.Factor(A, tol=tol, leaf_size=32, beta=16, h_sw=h_sw, dtype=dtype, seed=2)
    b = A.load(torch.tensor(pr.f, device=dev))
    return hx, A, P, b, fem.assemble_helmholtz(N, om, s)


@pytest.mark.parametrize("N,om,h_sw,dtype", [(33, 8.0, 1, "c128"), (65, 16.0, 2, "c128"),
                                              (65, 16.0, 2, "c64"), (129, 32.0, 3, "c128")])
def test_matrix_free_factor_solves(N, om, h_sw, dtype):
    hx, A, P, b, Ao = _solve_case(N, om, h_sw, 1e-6, dtype)
    st = P.stats()
    assert st["n_hss_nodes"] > 0 and st["n_compressed"] > 0
    if dtype == "c128":
        assert st["max_estimate"] <= 1e-6 and st["n_above_tol"] == 0
    x, stats = hx.gmres_solve(A, P, b, m=50, tol=1e-8, flexible=dtype == "c64")
    xo = x.cpu().numpy()
    bo = b.cpu().numpy()
    fe = exact.factor_exact(Ao, nd.build_nd(N, 32, 16), keep_S=False)
    xe = fe.apply(bo)
    for r in range(bo.shape[1]):
        assert stats[r]["converged"] and stats[r]["iters"] <= 12, stats[r]
        assert np.linalg.norm(Ao @ xo[:, r] - bo[:, r]) <= 1e-8 * np.linalg.norm(bo[:, r])
        assert np.linalg.norm(xo[:, r] - xe[:, r]) <= 1e-6 * np.linalg.norm(xe[:, r])
    # the transposed apply is the same map (complex symmetric factors), up
    # to the rounding of the factor's precision in the dense nodes' kernels
    y = P.apply(b).cpu().numpy()
    yt = P.apply(b, trans=True).cpu().numpy()
    assert np.linalg.norm(y - yt) <= (1e-12 if dtype == "c128" else 1e-5) * np.linalg.norm(y)


@pytest.mark.parametrize("N,om,h_sw", [(33, 8.0, 1), (65, 16.0, 2)])
def test_tolerance_to_zero_approaches_inverse(N, om, h_sw):
    """||P^-1 A x - x|| / ||x|| falls with the tolerance (no HSS step drops a term)."""
    dev = _dev()
    hx = _hssx()
    s = np.ones(N * N)
    A = hx.Operator(N, om, s)
    x = np.random.default_rng(5).standard_normal((N * N, 2)) + 0.5j
    xd = torch.tensor(x, device=dev)
    Ax = A.matvec(xd)
    errs = []
    for tol in (1e-4, 1e-7, 1e-10):
        P = hx.Factor(A, tol=tol, leaf_size=32, beta=16, h_sw=h_sw, seed=1)
        assert P.stats()["n_hss_nodes"] > 0
        y = P.apply(Ax).cpu().numpy()
        errs.append(np.linalg.norm(y - x) / np.linalg.norm(x))
    assert errs[2] <= 1e-6, errs
    assert errs[0] > errs[1] > errs[2], errs


def test_schur_complements_against_exact():
    """Compressed S(sigma) of HSS-class nodes against the oracle's exact
    Schur complements of the same boxes."""
    N, om, h_sw, tol = 65, 16.0, 1, 1e-8
    _dev()
    hx = _hssx()
    s = np.ones(N * N)
    A = hx.Operator(N, om, s)
    P = hx.Factor(A, tol=tol, leaf_size=32, beta=16, h_sw=h_sw, seed=1)
    Ao = fem.assemble_helmholtz(N, om, s)
    t = nd.build_nd(N, 32, 16)
    fe = exact.factor_exact(Ao, t)
    info = P.tree()
    checked = 0
    for k, bx in enumerate(t.boxes):
        if bx.is_leaf or bx.B.size == 0 or bx.height <= h_sw:
            continue
        S = P.schur(k, bx.B.size)
        err = np.linalg.norm(S - fe.S[k]) / np.linalg.norm(fe.S[k])
        assert err <= 1e3 * tol, (k, err)
        checked += 1
    assert checked > 0


def test_factor_cost_below_exact():
    """On the 263k-DOF grid's family (N = 257 here, the same rules), the
    HSS factorization's nominal flops and apply bytes are below the exact
    multifrontal factorization's."""
    N, om = 257, 50.0
    _dev()
    hx = _hssx()
    A = hx.Operator(N, om, np.ones(N * N))
    P = hx.Factor(A, tol=1e-6, leaf_size=32, beta=16, h_sw=4, dtype="c64", seed=1)
    st = P.stats()
    assert st["n_hss_nodes"] > 0
    assert st["factor_flops"] < st["exact_factor_flops"], st
    assert st["factor_bytes"] < st["exact_factor_bytes"], st
