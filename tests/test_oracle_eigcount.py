"""Pins of the oracle's eigenvalue count and dichotomy (Sec. 3.2, Sec. 4.1 step 2)."""
import numpy as np
import pytest

import oracle
import workloads as W


def _L(g):
    return oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, g.w)


def test_identity_block_gives_exact_trace():
    # R = I_N: <R, p(L~) R>_F = tr p(L~) = sum_l p(x_l)
    g = W.random_weighted(40, 0.2, 3)
    L = _L(g)
    lam, _ = oracle.dense_spectrum(L.toarray())
    lmax = lam[-1] * 1.01
    p = 60
    R = np.eye(g.n)
    mu = oracle.moments(L, lmax, p, R)
    for lc in (0.1 * lmax, 0.4 * lmax, 0.77 * lmax):
        a = oracle.cheb_coeffs(lc, lmax, p)
        tr = float(np.sum(oracle.cheb_eval(a, 2 * lam / lmax - 1)))
        assert oracle.eigcount_from_moments(mu, lc, lmax) == pytest.approx(tr, rel=1e-11, abs=1e-11)
        assert oracle.eigcount_literal(L, lmax, lc, p, R) == pytest.approx(tr, rel=1e-11, abs=1e-11)


def test_moments_route_equals_literal_route():
    g = W.workload_graph(1)
    L = _L(g)
    lmax = 31.0
    R = W.signals(g.n, 32, 5)[1]
    mu = oracle.moments(L, lmax, 50, R)
    for lc in (1.0, 5.0, 12.5):
        assert oracle.eigcount_from_moments(mu, lc, lmax) == pytest.approx(
            oracle.eigcount_literal(L, lmax, lc, 50, R), rel=1e-12, abs=1e-10)


def test_hutchinson_mean_and_variance():
    # E<R, p R> = tr p(L~);  Var = 2 sum_l p(x_l)^2 / R for Gaussian R with variance 1/R
    g = W.random_weighted(60, 0.1, 8)
    L = _L(g)
    lam, chi = oracle.dense_spectrum(L.toarray())
    lmax = lam[-1] * 1.01
    p, r = 40, 4
    lc = 0.3 * lmax
    a = oracle.cheb_coeffs(lc, lmax, p)
    px = oracle.cheb_eval(a, 2 * lam / lmax - 1)
    tr = px.sum()
    var = 2 * np.sum(px ** 2) / r
    vals = []
    for s in range(300):
        R = W.signals_f64(g.n, r, 1000 + s)
        vals.append(float(np.sum(R * oracle.dense_filter(lam, chi, lmax, a, R))))
    vals = np.array(vals)
    assert abs(vals.mean() - tr) < 3 * np.sqrt(var / len(vals))
    assert 0.7 * var < vals.var() < 1.3 * var


def test_large_gap_count_and_dichotomy():
    # k cliques joined by single edges: k small eigenvalues then a gap up to ~m
    k, m = 5, 12
    g = W.cliques(k, m, bridges=True)
    L = _L(g)
    lam, _ = oracle.dense_spectrum(L.toarray())
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, g.w)
    lmax = oracle.lmax_estimate(L, s, W.start_vector(g.n, 1), 100)
    assert lam[k] - lam[k - 1] > 5
    R = np.eye(g.n)  # exact trace: count is sum_l p(x_l)
    p = 120
    for lc in (0.5 * (lam[k - 1] + lam[k]),):
        c = oracle.eigcount_from_moments(oracle.moments(L, lmax, p, R), lc, lmax)
        assert round(c) == oracle.exact_count(lam, lc) == k
    est, traj = oracle.dichotomy_moments(L, lmax, k, p, 12, R)
    assert lam[k - 1] < est < lam[k]
    assert traj.shape == (12, 2)
    # the trajectory halves the bracket every step
    widths = [lmax / 2 ** (s + 1) for s in range(12)]
    mids = traj[:, 0]
    assert mids[0] == pytest.approx(lmax / 2)
    assert all(abs(mids[s + 1] - mids[s]) == pytest.approx(widths[s + 1]) for s in range(11))


def test_dichotomy_literal_equals_moments_branching():
    g = W.workload_graph(1)
    L = _L(g)
    lmax = 31.0
    R = W.signals(g.n, 32, 9)[1]
    e1, t1 = oracle.dichotomy_moments(L, lmax, 10, 50, 12, R)
    e2, t2 = oracle.dichotomy_literal(L, lmax, 10, 50, 12, R)
    assert e1 == e2
    np.testing.assert_allclose(t1, t2, rtol=1e-11, atol=1e-10)
