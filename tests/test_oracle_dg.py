"""Pins of the oracle's SIPG-P2 Helmholtz assembly (IPDG of Sec. 4.1-4.2,
symmetric variant) against facts that do not come from the oracle: the
block-pattern count, exact energies of continuous quadratics, the penalty and
consistency terms on element indicators, the exact mass, and the
third-order convergence of a manufactured plane wave."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem_dg


def _interp(Nc, fn):
    xy = fem_dg.dof_coords(Nc)
    return fn(xy[:, 0], xy[:, 1])


@pytest.mark.parametrize("Nc", [1, 2, 5])
def test_pattern_and_bitwise_symmetry(Nc):
    rng = np.random.default_rng(Nc)
    A = fem_dg.assemble_dg(Nc, 7.0, 0.5 + rng.random((Nc + 1) ** 2))
    assert A.nnz == fem_dg.dg_nnz(Nc)
    assert (A != A.T).nnz == 0
    if Nc == 5:
        assert fem_dg.dg_nnz(256) == 18837504


def test_continuous_quadratics_energy_exact():
    """For continuous u, v jumps vanish, so at omega = 0 the form reduces to
    int grad u . grad v; P2 holds global quadratics exactly.  Integrals by
    hand: grad(x^2).grad(xy) = 2xy -> 1/2; grad(x+2y).grad(y^2-x) = -1 + 4y
    -> 1; grad(xy).grad(xy) = x^2 + y^2 -> 2/3."""
    Nc = 4
    A = fem_dg.assemble_dg(Nc, 0.0)
    cases = [(lambda x, y: x * x, lambda x, y: x * y, 0.5),
             (lambda x, y: x + 2 * y, lambda x, y: y * y - x, 1.0),
             (lambda x, y: x * y, lambda x, y: x * y, 2.0 / 3.0)]
    for fu, fv, ref in cases:
        u, v = _interp(Nc, fu), _interp(Nc, fv)
        val = u @ (A @ v)
        assert val.real == pytest.approx(ref, rel=1e-12)
        assert abs(val.imag) < 1e-13


def test_mass_exact_for_quadratics():
    Nc = 3
    M = fem_dg.mass_matrix_dg(Nc)
    u = _interp(Nc, lambda x, y: 1 + x - y * y)
    v = _interp(Nc, lambda x, y: x * y + 2)
    # int (1 + x - y^2)(xy + 2) over the unit square, expanded by hand:
    # xy + x^2 y - x y^3 + 2 + 2x - 2y^2 -> 1/4 + 1/6 - 1/8 + 2 + 1 - 2/3
    ref = 0.25 + 1.0 / 6.0 - 0.125 + 2.0 + 1.0 - 2.0 / 3.0
    assert u @ (M @ v) == pytest.approx(ref, rel=1e-13)
    assert M.nnz == 36 * 2 * Nc * Nc                  # block diagonal


def test_penalty_on_element_indicators():
    """Piecewise constants have zero gradient: a(1_e, 1_e) = sum over e's
    interior faces of tau_F |F| = 10 p^2 = 40 each, and a(1_e, 1_e') = -40
    for face neighbours, 0 otherwise (omega = 0)."""
    Nc = 4
    A = fem_dg.assemble_dg(Nc, 0.0)
    ind = lambda e: np.repeat(np.eye(2 * Nc * Nc)[e], 6)  # noqa: E731
    interior = 2 * (1 * Nc + 1)            # lower triangle of cell (1,1): 3 interior faces
    west = 2 * (2 * Nc + 0) + 1            # upper triangle of cell (0,2): west face on the boundary
    assert ind(interior) @ (A @ ind(interior)) == pytest.approx(120.0, rel=1e-13)
    assert ind(west) @ (A @ ind(west)) == pytest.approx(80.0, rel=1e-13)
    assert ind(interior) @ (A @ ind(interior + 1)) == pytest.approx(-40.0, rel=1e-13)
    assert abs(ind(interior) @ (A @ ind(interior + 2))) < 1e-13


def test_consistency_term_sign():
    """a(x, 1_e) = - sum_{interior faces of e} int_F n_out,x: zero inside the
    domain and -h for an element whose west face lies on the boundary."""
    Nc = 4
    h = 1.0 / Nc
    A = fem_dg.assemble_dg(Nc, 0.0)
    x = _interp(Nc, lambda x, y: x)
    ind = lambda e: np.repeat(np.eye(2 * Nc * Nc)[e], 6)  # noqa: E731
    assert abs(ind(2 * (1 * Nc + 1)) @ (A @ x)) < 1e-13
    assert (ind(2 * (2 * Nc) + 1) @ (A @ x)).real == pytest.approx(-h, rel=1e-12)
    east = 2 * (2 * Nc + Nc - 1)           # lower triangle of the last column: east face outside
    assert (ind(east) @ (A @ x)).real == pytest.approx(h, rel=1e-12)


def _plane_wave_error(Nc, k, theta):
    """Nodal RMS error for u = exp(i k d.x) with Robin data g = d_n u - i k u
    on every side, b_i = int_boundary g phi_i by 4-point Gauss per face."""
    d = np.array([np.cos(theta), np.sin(theta)])
    A = fem_dg.assemble_dg(Nc, k)
    xy = fem_dg.dof_coords(Nc)
    u = np.exp(1j * k * (xy @ d))
    V, _ = fem_dg.elements(Nc)
    _, bnd = fem_dg.faces(Nc)
    t, w = np.polynomial.legendre.leggauss(4)
    t, w = (t + 1) / 2, w / 2
    b = np.zeros(A.shape[0], dtype=complex)
    edges = ((0, 1), (1, 2), (2, 0))
    for e, f in bnd:
        ps, pe = V[e, edges[f][0]], V[e, edges[f][1]]
        dv = pe - ps
        L = np.hypot(*dv)
        nrm = np.array([dv[1], -dv[0]]) / L
        pts = ps[None, :] + t[:, None] * dv[None, :]
        g = 1j * k * (nrm @ d - 1.0) * np.exp(1j * k * (pts @ d))
        phi, _ = fem_dg.basis(V[e:e + 1], pts[None])
        b[6 * e:6 * e + 6] += L * (w * g) @ phi[0]
    uh = spla.spsolve(A.tocsc(), b)
    return np.sqrt(np.mean(np.abs(uh - u) ** 2))


def test_plane_wave_third_order():
    errs = [_plane_wave_error(Nc, 4.0, np.pi / 6) for Nc in (4, 8, 16, 32)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates[1:] > 2.7) and np.all(rates < 3.6), (errs, rates)


def test_variable_slowness_scales():
    Nc = 3
    c = 1.7
    A1 = fem_dg.assemble_dg(Nc, 3.0, np.full((Nc + 1) ** 2, c))
    A2 = fem_dg.assemble_dg(Nc, 3.0 * c)
    assert abs(A1 - A2).max() < 1e-12


# ---------------------------------------------------------------- P1, Dirichlet
# The scaling study of Sec. 4.6 runs IPDG with p = 1 and u = 0 on the whole
# boundary (Sec. 4.1-4.2); the pins below fix the P1 basis and the boundary
# terms by closed forms and by the second-order convergence of a
# manufactured solution.

def _ind1(Nc, e):
    return np.repeat(np.eye(2 * Nc * Nc)[e], 3)


@pytest.mark.parametrize("Nc", [1, 2, 5])
def test_p1_dirichlet_pattern_and_symmetry(Nc):
    rng = np.random.default_rng(Nc)
    A = fem_dg.assemble_dg(Nc, 7.0, 0.5 + rng.random((Nc + 1) ** 2), deg=1, bc="dirichlet")
    assert A.shape == (6 * Nc * Nc, 6 * Nc * Nc)
    assert A.nnz == fem_dg.dg_nnz(Nc, 1)
    assert (A != A.T).nnz == 0
    assert abs(A.imag).max() == 0.0          # real operator: no absorbing term


def test_p1_dirichlet_linear_energies():
    """Continuous linear u, v have no interior jumps; by hand on the unit
    square with tau = 10 / h on the boundary faces:
    a(x, y) = 0 (volume) + 0 (consistency) + tau int_boundary x y = 10 Nc;
    a(x, x) = 1 - 2 int_{x=1} 1 + tau (1 + 1/3 + 1/3) = -1 + 50 Nc / 3."""
    Nc = 4
    A = fem_dg.assemble_dg(Nc, 0.0, deg=1, bc="dirichlet")
    xy = fem_dg.dof_coords(Nc, 1)
    x, y = xy[:, 0], xy[:, 1]
    assert (x @ (A @ y)).real == pytest.approx(10.0 * Nc, rel=1e-12)
    assert (x @ (A @ x)).real == pytest.approx(-1.0 + 50.0 * Nc / 3.0, rel=1e-12)


def test_p1_dirichlet_penalty_on_indicators():
    """Piecewise constants: every face of an element, interior or on the
    Dirichlet boundary, adds tau |F| = 10 p^2 = 10, so a(1_e, 1_e) = 30 for
    every e; face neighbours couple with -10 (omega = 0)."""
    Nc = 4
    A = fem_dg.assemble_dg(Nc, 0.0, deg=1, bc="dirichlet")
    for e in (0, 2 * (1 * Nc + 1), 2 * (2 * Nc) + 1, 2 * Nc * Nc - 1):
        assert _ind1(Nc, e) @ (A @ _ind1(Nc, e)) == pytest.approx(30.0, rel=1e-13)
    e = 2 * (1 * Nc + 1)
    assert _ind1(Nc, e) @ (A @ _ind1(Nc, e + 1)) == pytest.approx(-10.0, rel=1e-13)
    assert abs(_ind1(Nc, e) @ (A @ _ind1(Nc, e + 2))) < 1e-13


def test_p1_dirichlet_consistency_signs():
    """a(x, 1_e): zero inside; zero for a triangle with its face on x = 0
    (the boundary consistency term +h cancels the interior faces' -h); and
    -h + (h - h) + tau h = 10 for a triangle with its face on x = 1."""
    Nc = 4
    A = fem_dg.assemble_dg(Nc, 0.0, deg=1, bc="dirichlet")
    x = fem_dg.dof_coords(Nc, 1)[:, 0]
    assert abs(_ind1(Nc, 2 * (1 * Nc + 1)) @ (A @ x)) < 1e-13
    assert abs(_ind1(Nc, 2 * (2 * Nc) + 1) @ (A @ x)) < 1e-13
    east = 2 * (2 * Nc + Nc - 1)
    assert (_ind1(Nc, east) @ (A @ x)).real == pytest.approx(10.0, rel=1e-12)


def _p1_manufactured_error(Nc, kappa):
    """Nodal RMS error for u = sin(pi x) sin(pi y) (zero on the boundary),
    f = (2 pi^2 - kappa^2) u, b_i = int f phi_i by the 16-point rule."""
    A = fem_dg.assemble_dg(Nc, kappa, deg=1, bc="dirichlet")
    V, _ = fem_dg.elements(Nc)
    pts, w, _ = fem_dg._tri_quad(V)
    phi, _ = fem_dg.basis(V, pts, 1)
    f = (2 * np.pi ** 2 - kappa ** 2) * np.sin(np.pi * pts[..., 0]) * np.sin(np.pi * pts[..., 1])
    b = np.einsum("eq,eqa->ea", w * f, phi).ravel() + 0j
    uh = spla.spsolve(A.tocsc(), b)
    xy = fem_dg.dof_coords(Nc, 1)
    u = np.sin(np.pi * xy[:, 0]) * np.sin(np.pi * xy[:, 1])
    return np.sqrt(np.mean(np.abs(uh - u) ** 2))


@pytest.mark.parametrize("kappa,grids", [(0.0, (8, 16, 32, 64)), (10.0, (16, 32, 64, 128))])
def test_p1_dirichlet_second_order(kappa, grids):
    """Every refinement gains at least second order less a margin; the mean
    rate over the range is second order (the Helmholtz error mixes the
    pollution term into single steps, so only the mean is held from above)."""
    errs = np.array([_p1_manufactured_error(Nc, kappa) for Nc in grids])
    rates = np.log2(errs[:-1] / errs[1:])
    mean = np.log2(errs[0] / errs[-1]) / (len(grids) - 1)
    assert np.all(rates > 1.8) and 1.85 < mean < 2.3, (errs, rates, mean)
