"""Pins of the oracle's Laplacian (Sec. 2.1) and lambda_N estimate (Sec. 4.1 step 1)."""
import os

import numpy as np
import pytest
import scipy.sparse.csgraph as csgraph

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "laplacian_spectra.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        out[parts[0]] = (int(parts[1]), np.array([float(x) for x in parts[2:]]))
    return out


NAMED = {
    "complete5": lambda: W.complete(5),
    "cycle6": lambda: W.cycle(6),
    "cycle4": lambda: W.cycle(4),
    "path3": lambda: W.path(3),
    "path4": lambda: W.path(4),
    "star5": lambda: W.star(5),
    "cliques3x4": lambda: W.cliques(3, 4),
}


def _L(g):
    return oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, g.w)


@pytest.mark.parametrize("name", sorted(NAMED))
def test_golden_spectra(name):
    n, lam_ref = _golden()[name]
    g = NAMED[name]()
    assert g.n == n
    lam, chi = oracle.dense_spectrum(_L(g).toarray())
    np.testing.assert_allclose(lam, lam_ref, atol=1e-12)


@pytest.mark.parametrize("n", [5, 8, 13])
def test_closed_form_cycle_path(n):
    m = np.arange(n)
    lam_c = np.sort(2 - 2 * np.cos(2 * np.pi * m / n))
    lam_p = np.sort(2 - 2 * np.cos(np.pi * m / n))
    np.testing.assert_allclose(oracle.dense_spectrum(_L(W.cycle(n)).toarray())[0], lam_c, atol=1e-12)
    np.testing.assert_allclose(oracle.dense_spectrum(_L(W.path(n)).toarray())[0], lam_p, atol=1e-12)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_laplacian_invariants(seed):
    g = W.random_weighted(40, 0.15, seed, isolated=3)
    oracle.check_graph(g.n, g.row_ptr, g.col_idx, g.w)
    L = _L(g).toarray()
    np.testing.assert_allclose(L @ np.ones(g.n), 0, atol=1e-12)
    np.testing.assert_array_equal(L, L.T)
    lam, _ = oracle.dense_spectrum(L)
    assert lam[0] >= -1e-12 * lam[-1]
    ncomp = csgraph.connected_components(_L(g) != 0, directed=False)[0]
    assert int(np.sum(lam < 1e-9 * lam[-1])) == ncomp
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, g.w)
    np.testing.assert_allclose(np.diag(L), s, rtol=1e-15)


def test_check_graph_rejects():
    g = W.cycle(5)
    bad = g.col_idx.copy()
    bad[0] = 0  # self-loop on row 0
    with pytest.raises(ValueError):
        oracle.check_graph(g.n, g.row_ptr, bad, g.w)
    w = g.w.copy()
    w[0] = -1
    with pytest.raises(ValueError):
        oracle.check_graph(g.n, g.row_ptr, g.col_idx, w)
    w = g.w.copy()
    w[0] = 2.0  # breaks W_ij = W_ji
    with pytest.raises(ValueError):
        oracle.check_graph(g.n, g.row_ptr, g.col_idx, w)


@pytest.mark.parametrize("make", [lambda: W.complete(7), lambda: W.cycle(10), lambda: W.path(9),
                                  lambda: W.star(6), lambda: W.random_weighted(60, 0.1, 4, isolated=2),
                                  lambda: W.workload_graph(1)])
def test_lanczos_lmax(make):
    g = make()
    L = _L(g)
    lam, _ = oracle.dense_spectrum(L.toarray())
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, g.w)
    v0 = W.start_vector(g.n, 11)
    theta = oracle.lanczos_lmax(L, v0, 200, s.max())
    # Ritz values are lower bounds and the largest converges to lambda_N
    assert theta <= lam[-1] * (1 + 1e-12)
    assert theta >= lam[-1] * (1 - 1e-9)
    est = oracle.lmax_estimate(L, s, v0, 200)
    assert lam[-1] <= est <= 1.0101 * lam[-1]
    # Rayleigh quotient at a unit vector and Gershgorin
    assert s.max() <= lam[-1] * (1 + 1e-12) and lam[-1] <= 2 * s.max() * (1 + 1e-12)


def test_lmax_unweighted_lower_bound():
    # for unit weights lambda_N >= d_max + 1 (any graph with an edge)
    g = W.workload_graph(1)
    L = _L(g)
    lam, _ = oracle.dense_spectrum(L.toarray())
    dmax = np.diff(g.row_ptr).max()
    assert lam[-1] >= dmax + 1 - 1e-9
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, g.w)
    est = oracle.lmax_estimate(L, s, W.start_vector(g.n, 3), 60)
    assert lam[-1] <= est <= 1.02 * lam[-1]


@pytest.mark.parametrize("n", [3, 7, 12])
def test_normalized_laplacian_closed_forms(n):
    # complete graph K_n: eigenvalues 0 and n/(n-1) (n-1 times)
    g = W.complete(n)
    lam = np.linalg.eigvalsh(oracle.laplacian_normalized(g.n, g.row_ptr, g.col_idx).toarray())
    np.testing.assert_allclose(lam, [0.0] + [n / (n - 1)] * (n - 1), atol=1e-12)
    # cycle C_n: 1 - cos(2 pi k / n)
    g = W.cycle(n)
    lam = np.linalg.eigvalsh(oracle.laplacian_normalized(g.n, g.row_ptr, g.col_idx).toarray())
    ref = np.sort(1.0 - np.cos(2 * np.pi * np.arange(n) / n))
    np.testing.assert_allclose(lam, ref, atol=1e-12)


def test_normalized_laplacian_invariants():
    rng = np.random.default_rng(3)
    g = W.random_weighted(60, 0.1, 4, isolated=3)
    Ln = oracle.laplacian_normalized(g.n, g.row_ptr, g.col_idx, g.w).toarray()
    lam = np.linalg.eigvalsh(Ln)
    assert lam.min() > -1e-12 and lam.max() < 2 + 1e-12
    np.testing.assert_allclose(Ln, Ln.T, atol=0)
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, g.w)
    np.testing.assert_allclose(Ln @ np.sqrt(s), 0.0, atol=1e-12)
    # isolated nodes: rows of the identity (eigenvalue 1)
    for i in range(g.n - 3, g.n):
        e = np.zeros(g.n)
        e[i] = 1
        np.testing.assert_array_equal(Ln[i], e)
    # bipartite (even cycle, path) graphs reach the bound 2
    for gb in (W.cycle(10), W.path(9)):
        lb = np.linalg.eigvalsh(oracle.laplacian_normalized(gb.n, gb.row_ptr, gb.col_idx).toarray())
        assert abs(lb.max() - 2.0) < 1e-12
    del rng
