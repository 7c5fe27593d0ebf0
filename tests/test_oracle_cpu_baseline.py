"""The plain-C FP64 CPU baseline equals the NumPy oracle recurrence."""
import numpy as np
import pytest

import oracle
import oracle.cpu_baseline as cb
import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _built():
    cb.ensure_built()


@pytest.mark.parametrize("p", [0, 1, 2, 50])
@pytest.mark.parametrize("weighted", [False, True])
def test_c_baseline_matches_oracle(p, weighted):
    g = W.random_weighted(300, 0.03, 4, isolated=5) if weighted else W.workload_graph(1)
    w = g.w.astype(np.float64) if weighted else None
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, w)
    lmax = 1.01 * oracle.lambda_max_exact(L)
    R = W.signals(g.n, 12, 3)[1]
    a = oracle.cheb_coeffs(0.2 * lmax, lmax, p)
    Y1 = oracle.cheb_filter(L, lmax, a, R)
    Y2 = cb.cheb_filter(g.n, g.row_ptr, g.col_idx, w, lmax, a, R)
    assert np.linalg.norm(Y1 - Y2) <= 1e-13 * np.linalg.norm(Y1) + 1e-300


@pytest.mark.parametrize("p", [0, 1, 2, 37])
@pytest.mark.parametrize("weighted", [False, True])
def test_c_moments_match_oracle(p, weighted):
    g = W.random_weighted(250, 0.04, 7, isolated=3) if weighted else W.workload_graph(1)
    w = g.w.astype(np.float64) if weighted else None
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, w)
    lmax = 1.01 * oracle.lambda_max_exact(L)
    R = W.signals(g.n, 5, 9)[1]
    mu1 = oracle.moments(L, lmax, p, R)
    mu2 = cb.cheb_moments(g.n, g.row_ptr, g.col_idx, w, lmax, p, R)
    np.testing.assert_allclose(mu2, mu1, rtol=0, atol=1e-12 * abs(mu1[0]))
