"""The plain-C FP64 CPU baseline equals the NumPy oracle recurrence."""
import os

import numpy as np
import pytest

import oracle
import oracle.cpu_baseline as cb
import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(cb.LIB):
        cb.build()


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
