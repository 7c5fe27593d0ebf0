"""GPU parity of the order-selection table (note on the choice of m, Sec. 2.4)
against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import order
import paper_1509_08863_amd as asc

from gpu_util import DEV, host

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
