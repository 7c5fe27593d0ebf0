"""GPU parity of the order-selection table (note on the choice of m, Sec. 2.4)
against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from oracle import order
import workloads as W
import paper_1509_08863_amd as asc

from gpu_util import DEV, host, upload_graph, block_f32, scalar, rel_fro

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("band,G", [(0.01, 1025), (0.0, 257), (0.002, 4097)])
def test_order_table_matches_oracle(band, G):
    rho = np.array([0.003, 0.02, 0.13, 0.5, 0.87])
    delta = np.array([0.3, 0.1, 0.03])
    m_max = 300
    ms, err = asc.order_table(torch.tensor(rho, device=DEV), torch.tensor(delta, device=DEV), band, m_max, G)
    ms, err = host(ms), host(err)
    for q, r in enumerate(rho):
        ref = order.order_errors(r, m_max, band, G)
        np.testing.assert_allclose(err[q], ref, rtol=1e-9, atol=1e-11)
        for d, dl in enumerate(delta):
            assert ms[q, d] == order.m_star(r, dl, m_max, band, G), (r, dl)


def test_order_table_undamped_and_limits():
    rho = torch.tensor([0.3], dtype=torch.float64, device=DEV)
    delta = torch.tensor([0.05, 2.0], dtype=torch.float64, device=DEV)
    ms, err = asc.order_table(rho, delta, 0.002, 200, 1025, jackson=False)
    ref = order.order_errors(0.3, 200, 0.002, 1025, jackson=False)
    np.testing.assert_allclose(host(err)[0], ref, rtol=1e-9, atol=1e-11)
    assert host(ms)[0, 0] == 201 and host(ms)[0, 1] == 1


def test_order_for_relative_band():
    lc, lmax = 0.5e-3 * 20.0, 20.0
    m = asc.order_for(lc, lmax, delta=0.1, band_rel=0.5, m_max=1000, grid=2049)
    rho = lc / lmax
    assert m == order.m_star(rho, 0.1, 1000, 0.5 * rho, 2049)
    assert 100 < m < 1000


def test_lambda_k_filter_with_the_order_from_the_table():
    # the table feeds p (note on m, Sec. 2.4): lambda_k from the moment
    # dichotomy, p = m*(lambda_k / lmax; delta) with a band of half the cut-off,
    # then the order-p filter; checked against the oracle's m* and filter
    g = W.workload_graph(1)
    G = upload_graph(g)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, None)
    lmax = oracle.lmax_estimate(L, oracle.strength(g.n, g.row_ptr, g.col_idx, None), W.start_vector(g.n, 1), 60)
    Rs, R64 = W.signals(g.n, 16, 4)
    k, p_count, steps = 10, 50, 12
    Y, lam, traj, p = asc.lambda_k_filter_auto(G, scalar(lmax), k, block_f32(Rs), delta=0.1, band_rel=0.5,
                                               p_count=p_count, steps=steps, m_max=2000)
    lam_h = float(host(lam)[0])
    rho = lam_h / lmax
    assert p == order.m_star(rho, 0.1, 2000, 0.5 * rho, 2049)
    print("lambda_k / lmax", rho, "order", p)
    a = oracle.cheb_coeffs(lam_h, lmax, p)
    assert rel_fro(host(Y), oracle.cheb_filter(L, lmax, a, R64)) <= 1e-5
    est, traj_ref = oracle.dichotomy_moments(L, lmax, k, p_count, steps, R64)
    if np.all(np.abs(traj_ref[:, 1] - (k - 0.5)) > 1e-3):
        assert lam_h == est
    with pytest.raises(ValueError):
        asc.lambda_k_filter_auto(G, scalar(lmax), k, block_f32(Rs), delta=1e-9, p_count=p_count, m_max=40)
