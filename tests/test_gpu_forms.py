"""GPU tests of the execution forms: the apply sweeps replayed as a captured
HIP graph, autotuned apply tiles, and the bf16 sampling precision form."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import exact, fem, nd  # noqa: E402
from synth import make_problem  # noqa: E402


def _hx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2105_07791_amd import hssx
    return hssx


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("nrhs", [1, 5])
def test_apply_graph_replays_match_eager(dtype, nrhs):
    """Every replay of the captured sweeps equals the eager apply bit for bit,
    with eager work and synchronisations between the replays."""
    hx = _hx()
    dev = torch.device("cuda:0")
    pr = make_problem("helmholtz_p1_65")
    A = hx.Operator(pr.N, pr.omega, pr.slowness)
    Pg = hx.Factor(A, tol=1e-6, h_sw=2, dtype=dtype, seed=4, apply_graph=True)
    Pe = hx.Factor(A, tol=1e-6, h_sw=2, dtype=dtype, seed=4, apply_graph=False)
    rng = np.random.default_rng(nrhs)
    for rep in range(4):
        x = rng.standard_normal((pr.n, nrhs)) + 1j * rng.standard_normal((pr.n, nrhs))
        xt = torch.tensor(x, device=dev)
        for trans in (False, True):
            yg = Pg.apply(xt, trans=trans)
            A.matvec(xt)                      # unrelated eager work in between
            torch.cuda.synchronize()
            ye = Pe.apply(xt, trans=trans)
            torch.cuda.synchronize()
            assert torch.equal(yg, ye), (rep, trans)


def test_autotuned_tiles_do_not_change_results():
    """Tile shapes only change the thread mapping, not the summation order."""
    hx = _hx()
    dev = torch.device("cuda:0")
    pr = make_problem("helmholtz_p1_65")
    A = hx.Operator(pr.N, pr.omega, pr.slowness)
    Pa = hx.Factor(A, tol=1e-6, h_sw=2, dtype="c64", seed=4, autotune=True)
    Pf = hx.Factor(A, tol=1e-6, h_sw=2, dtype="c64", seed=4, autotune=False)
    rng = np.random.default_rng(3)
    for nrhs in (1, 7, 64):
        x = torch.tensor(rng.standard_normal((pr.n, nrhs)) + 0j, device=dev)
        assert torch.equal(Pa.apply(x), Pf.apply(x))


def test_graph_apply_through_gmres_matches_oracle():
    hx = _hx()
    dev = torch.device("cuda:0")
    pr = make_problem("helmholtz_p1_65")
    A = hx.Operator(pr.N, pr.omega, pr.slowness)
    P = hx.Factor(A, tol=1e-6, h_sw=2, dtype="c64", apply_graph=True)
    b = A.load(torch.tensor(pr.f, device=dev))
    x, st = hx.gmres_solve(A, P, b, flexible=True)
    Ao = fem.assemble_helmholtz(pr.N, pr.omega, pr.slowness)
    bo = fem.mass_matrix(pr.N) @ pr.f + 0j
    xo = exact.factor_exact(Ao, nd.build_nd(pr.N, 32, 16), keep_S=False).apply(bo)
    xg = x.cpu().numpy().reshape(pr.n, -1)
    assert st[0]["converged"]
    assert np.linalg.norm(xg - xo) <= 1e-6 * np.linalg.norm(xo)


def test_bf16_sampling_form():
    """Sampling products on bf16 matrix cores (fp32 accumulation): the
    adaptive compression still meets its estimate at a tolerance above the
    bf16 rounding level, and flexible GMRES reaches the oracle solution."""
    hx = _hx()
    dev = torch.device("cuda:0")
    pr = make_problem("helmholtz_p1_65")
    A = hx.Operator(pr.N, pr.omega, pr.slowness)
    P16 = hx.Factor(A, tol=1e-2, h_sw=2, dtype="c64", seed=5, sample_bf16=True)
    P32 = hx.Factor(A, tol=1e-2, h_sw=2, dtype="c64", seed=5, sample_bf16=False)
    s16, s32 = P16.stats(), P32.stats()
    assert s16["n_compressed"] > 0
    assert s16["max_estimate"] <= 1e-2 and s16["max_rounds_used"] < 32
    assert s16["k_max"] <= 2 * max(s32["k_max"], 16)
    b = A.load(torch.tensor(pr.f, device=dev))
    y16 = P16.apply(b).cpu().numpy()
    y32 = P32.apply(b).cpu().numpy()
    assert np.linalg.norm(y16 - y32) <= 5e-2 * np.linalg.norm(y32)
    x, st = hx.gmres_solve(A, P16, b, flexible=True)
    Ao = fem.assemble_helmholtz(pr.N, pr.omega, pr.slowness)
    bo = fem.mass_matrix(pr.N) @ pr.f + 0j
    xo = exact.factor_exact(Ao, nd.build_nd(pr.N, 32, 16), keep_S=False).apply(bo)
    assert st[0]["converged"]
    assert np.linalg.norm(x.cpu().numpy().reshape(pr.n, -1) - xo) <= 1e-6 * np.linalg.norm(xo)


def test_bf16_sampling_needs_complex64():
    hx = _hx()
    from paper_2105_07791_amd._lib import HssxError
    pr = make_problem("helmholtz_p1_17")
    A = hx.Operator(pr.N, pr.omega, pr.slowness)
    with pytest.raises(HssxError):
        hx.Factor(A, dtype="c128", sample_bf16=True)


def test_split_bf16_sampling_reaches_fp32_quality():
    """Head/tail bf16 operands (three matrix-core products) sample accurately
    enough for the compression to certify 1e-4 with fp32-like ranks."""
    hx = _hx()
    dev = torch.device("cuda:0")
    pr = make_problem("helmholtz_p1_65")
    A = hx.Operator(pr.N, pr.omega, pr.slowness)
    Ps = hx.Factor(A, tol=1e-4, h_sw=2, dtype="c64", seed=5, sample_bf16=2)
    Pf = hx.Factor(A, tol=1e-4, h_sw=2, dtype="c64", seed=5, sample_bf16=0)
    ss, sf = Ps.stats(), Pf.stats()
    assert ss["max_estimate"] <= 1e-4 and ss["max_rounds_used"] < 32
    assert ss["k_max"] <= sf["k_max"] + 16
    b = A.load(torch.tensor(pr.f, device=dev))
    ys, yf = Ps.apply(b).cpu().numpy(), Pf.apply(b).cpu().numpy()
    assert np.linalg.norm(ys - yf) <= 1e-3 * np.linalg.norm(yf)
