"""Pins of the order-selection oracle (note on the choice of m, Sec. 2.4)."""
import numpy as np
import pytest

from oracle import order

G = 1025


@pytest.mark.parametrize("rho", [0.02, 0.13, 0.3, 0.45])
def test_mirror_symmetry(rho):
    # p for 1 - rho is 1 - p(-x): the error pattern is mirrored about x = 0
    e1 = order.order_errors(rho, 60, 0.02, G)
    e2 = order.order_errors(1.0 - rho, 60, 0.02, G)
    np.testing.assert_allclose(e1, e2, atol=1e-12)
    assert order.m_star(rho, 0.1, 200, 0.02, G) == order.m_star(1.0 - rho, 0.1, 200, 0.02, G)


def test_delta_one_needs_order_one():
    # Jackson-damped approximations of a step stay in [0, 1]
    for rho in (0.01, 0.2, 0.5, 0.9):
        assert order.m_star(rho, 1.0, 50, 0.0, G) == 1
        assert np.all(order.order_errors(rho, 40, 0.0, G) <= 1.0 + 1e-12)


def test_undamped_series_overshoots():
    # without damping the truncated series does not converge uniformly near
    # the jump (Gibbs): just outside a thin band the error stays large however
    # large m is
    e = order.order_errors(0.3, 200, 0.002, G, jackson=False)
    assert e[-1] > 0.05
    assert order.m_star(0.3, 0.05, 200, 0.002, G, jackson=False) == 201


def test_definition_and_monotonicity():
    rho, w, m_max = 0.1, 0.01, 400
    e = order.order_errors(rho, m_max, w, G)
    prev = None
    for delta in (0.3, 0.1, 0.05, 0.02):
        m = order.m_star(rho, delta, m_max, w, G)
        assert 1 <= m <= m_max
        assert e[m - 1] <= delta
        assert m == 1 or e[m - 2] > delta
        if prev is not None:
            assert m >= prev
        prev = m
    # a wider band never needs a higher order
    assert order.m_star(rho, 0.05, m_max, 0.02, G) <= order.m_star(rho, 0.05, m_max, 0.01, G)


def test_error_decays_like_inverse_cube():
    # at a fixed distance d from the jump the damped step's error is the tail
    # mass of the Jackson kernel beyond d, which falls like (m d)^-3: doubling
    # m divides it by about 8 (between 4 and 20 on this grid), and it never
    # stalls (the undamped series, by contrast, does not converge near a jump)
    e = order.order_errors(0.4, 800, 0.05, G)
    assert e[799] < e[399] < e[199] < e[99] < e[49]
    for m in (100, 200, 400, 800):
        assert 1 / 20 < e[m - 1] / e[m // 2 - 1] < 1 / 4
