"""Pins of the oracle HSS code: interpolative decomposition, the two
independent HSS evaluations (telescoping product vs. nested-basis expansion),
exact recovery of a known-rank HSS matrix by Algorithm A.1, error control on
exact Schur complements, the estimator's expectation (eq. 2.7), and the
counter-based generator's published known answers."""
import os

import numpy as np
import pytest

from oracle import exact, fem, hss, nd, rng

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLD, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = rng.philox4x32(*v[:6])
        assert [int(o) for o in out] == v[6:]


def test_gaussian_moments():
    g = rng.gaussian_block(11, 3, 400, 0, 500)
    assert abs(g.mean()) < 0.01
    assert abs(g.std() - 1.0) < 0.01
    assert abs(np.mean(g ** 4) - 3.0) < 0.05
    # counter-based: a column block is the same wherever it is drawn from
    assert np.array_equal(rng.gaussian_block(11, 3, 400, 100, 7), g[:, 100:107])


def test_interp_decomp_properties():
    r = np.random.default_rng(0)
    X = r.standard_normal((50, 6)) + 1j * r.standard_normal((50, 6))
    Y = r.standard_normal((6, 30))
    S = X @ Y                                        # rank 6
    U, J = hss.interp_decomp(S, 20, 1e-12)
    assert U.shape[1] == 6
    assert np.array_equal(U[J], np.eye(6))
    assert np.linalg.norm(U @ S[J] - S) < 1e-12 * np.linalg.norm(S)
    U2, J2 = hss.interp_decomp(S, 4)                 # rank-limited
    assert U2.shape[1] == 4 and np.array_equal(U2[J2], np.eye(4))


def _tree(N=65):
    t = nd.build_nd(N, 32, 16)
    return t, t.boxes[t.boxes[-1].lo].ctree


def test_matvec_equals_expansion():
    _, ct = _tree()
    H = hss.random_hss(ct, 5, seed=2)
    D = H.dense()
    X = np.random.default_rng(1).standard_normal((D.shape[0], 4))
    assert np.linalg.norm(H.matvec(X) - D @ X) < 1e-13 * np.linalg.norm(D @ X)
    assert np.linalg.norm(D - D.T) < 1e-13 * np.linalg.norm(D)


@pytest.mark.parametrize("k_true,seed", [(3, 0), (6, 1), (9, 2)])
def test_recovers_known_rank(k_true, seed):
    _, ct = _tree()
    H = hss.random_hss(ct, k_true, seed=seed)
    D = H.dense()
    H2 = hss.compress_adaptive(lambda X: D @ X, lambda I, J: D[np.ix_(I, J)],
                               ct, k0=k_true + 2, r=4, tol=1e-10, seed=seed)
    assert np.linalg.norm(H2.dense() - D) < 1e-11 * np.linalg.norm(D)
    assert H2.max_rank() <= k_true + 2


def test_rank_growth_when_k0_small():
    _, ct = _tree()
    H = hss.random_hss(ct, 10, seed=5)
    D = H.dense()
    H2 = hss.compress_adaptive(lambda X: D @ X, lambda I, J: D[np.ix_(I, J)],
                               ct, k0=2, r=4, tol=1e-10, seed=5)
    assert H2.rounds > 1 and H2.k_final >= 10
    assert np.linalg.norm(H2.dense() - D) < 1e-9 * np.linalg.norm(D)


def test_tolerance_on_exact_schur_complements():
    N = 65
    A = fem.assemble_helmholtz(N, 16.0)
    t = nd.build_nd(N, 32, 16)
    f = exact.factor_exact(A, t)
    big = sorted(range(len(t.boxes) - 1), key=lambda k: -t.boxes[k].B.size)[:6]
    for seed in range(3):
        for k in big:
            S = f.S[k]
            H = hss.compress_adaptive(lambda X: S @ X, lambda I, J: S[np.ix_(I, J)],
                                      t.boxes[k].ctree, tol=1e-6, seed=seed,
                                      instance=4 * k)
            err = np.linalg.norm(H.dense() - S) / np.linalg.norm(S)
            assert err <= 1e-6
            Hp = hss.compress_plain(S, t.boxes[k].ctree, 1e-6)
            assert np.linalg.norm(Hp.dense() - S) / np.linalg.norm(S) <= 1e-6


def test_estimator_expectation():
    """E ||E w||^2 = ||E||_F^2 for w with iid zero-mean unit-variance entries
    (eq. 2.7, Sec. 2.3)."""
    r = np.random.default_rng(4)
    E = r.standard_normal((40, 40)) + 1j * r.standard_normal((40, 40))
    W = rng.gaussian_block(1, 1, 40, 0, 20000)
    est = np.sum(np.abs(E @ W) ** 2) / W.shape[1]
    assert abs(est / np.linalg.norm(E) ** 2 - 1.0) < 0.03
