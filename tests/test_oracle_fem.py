"""Pins of the oracle's P1 Helmholtz assembly against closed forms and the
manufactured plane-wave rate (Sec. 4.2, eq. 4.2 with an absorbing boundary)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem


@pytest.mark.parametrize("N", [2, 5, 9, 65])
def test_pattern_and_bitwise_symmetry(N):
    A = fem.assemble_helmholtz(N, 3.0, np.linspace(0.5, 1.5, N * N))
    assert A.nnz == fem.stencil_nnz(N)
    assert (A != A.T).nnz == 0                      # bitwise complex symmetric
    if N == 65:
        assert A.nnz == 29057


def test_mass_stiffness_boundary_sums():
    N = 17
    h = 1.0 / (N - 1)
    K = fem.assemble_helmholtz(N, 0.0).real
    G = -(fem.assemble_helmholtz(N, 1.0) - fem.assemble_helmholtz(N, 0.0)
          + fem.mass_matrix(N)).imag
    M = fem.mass_matrix(N)
    assert abs(M.sum() - 1.0) < 1e-13               # area of the unit square
    assert np.abs(K @ np.ones(N * N)).max() < 1e-13  # constants in the kernel
    assert abs(G.sum() - 4.0) < 1e-13               # perimeter
    # interior rows: 5-point Laplacian (diagonal edges carry zero stiffness,
    # -cot(90deg)/2) and the P1 mass row h^2/2 on the diagonal, h^2/12 x 6
    i = 8 * N + 8
    krow = K[i].toarray().ravel()
    mrow = M[i].toarray().ravel()
    nb = [i - N - 1, i - N, i - 1, i + 1, i + N, i + N + 1]
    assert krow[i] == pytest.approx(4.0, abs=1e-14)
    assert np.allclose(krow[[i - N, i - 1, i + 1, i + N]], -1.0, atol=1e-14)
    assert np.allclose(krow[[i - N - 1, i + N + 1]], 0.0, atol=1e-14)
    assert mrow[i] == pytest.approx(h * h / 2, rel=1e-13)
    assert np.allclose(mrow[nb], h * h / 12, rtol=1e-13)
    assert np.count_nonzero(mrow) == 7


def test_two_triangle_closed_form():
    """One cell, h = 1, triangles (0,1,3), (0,3,2).  Entries written out from
    int_T l_a l_b l_c = 2|T| a!b!c!/(a+b+c+2)! with |T| = 1/2."""
    s = np.array([0.7, 1.3, 0.9, 1.1])
    w = s * s
    om = 2.5
    A = fem.assemble_helmholtz(2, om, s).toarray()
    # M[w](0,0): both triangles contain node 0
    m00 = w[0] / 10 + (w[1] + 2 * w[3] + w[2]) / 60
    # M[w](0,3): shared edge (0,3) in both triangles; third vertices 1 and 2
    m03 = 2 * (w[0] + w[3]) / 60 + (w[1] + w[2]) / 120
    # boundary: node 0 touches edges (0,1) and (0,2); G(0,0) = sum s_l int l_l l0^2
    g00 = (s[0] / 4 + s[1] / 12) + (s[0] / 4 + s[2] / 12)
    g03 = 0.0                                     # (0,3) is the diagonal, interior
    k00 = 1.0                                     # K row of node 0: [1, -1/2, -1/2, 0]
    assert A[0, 0] == pytest.approx(k00 - om ** 2 * m00 - 1j * om * g00, rel=1e-14)
    assert A[0, 3] == pytest.approx(0.0 - om ** 2 * m03 - 1j * om * g03, rel=1e-14)


def _plane_wave_error(N, k, theta):
    """Nodal RMS error of the P1 solution for u = exp(i k d.x) with Robin data
    g = d_n u - i k u on every side (b_i = int_boundary g phi_i)."""
    h = 1.0 / (N - 1)
    d = np.array([np.cos(theta), np.sin(theta)])
    x = np.tile(np.arange(N) * h, N)
    y = np.repeat(np.arange(N) * h, N)
    u = np.exp(1j * k * (d[0] * x + d[1] * y))
    A = fem.assemble_helmholtz(N, k)
    b = np.zeros(N * N, dtype=complex)
    edges = fem.boundary_edges(N)
    normals = np.repeat(np.array([[0, -1], [1, 0], [0, 1], [-1, 0]]), N - 1, axis=0)
    for (a, c), nrm in zip(edges, normals):
        fac = 1j * k * (nrm @ d - 1.0)              # g = i k (n.d - 1) u
        ga, gc = fac * u[a], fac * u[c]
        b[a] += h / 6 * (2 * ga + gc)
        b[c] += h / 6 * (ga + 2 * gc)
    uh = spla.spsolve(A.tocsc(), b)
    return np.sqrt(np.mean(np.abs(uh - u) ** 2))


def test_plane_wave_second_order():
    errs = [_plane_wave_error(N, 4.0, np.pi / 6) for N in (17, 33, 65, 129)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.2), (errs, rates)


def test_variable_slowness_scales():
    N = 9
    c = 1.7
    A1 = fem.assemble_helmholtz(N, 3.0, np.full(N * N, c))
    A2 = fem.assemble_helmholtz(N, 3.0 * c)       # k = omega*s is what enters
    assert abs(A1 - A2).max() < 1e-12
