"""Pins of the order-selection oracle (note on the choice of m, Sec. 2.4)."""
import numpy as np
import pytest

from oracle import cheb, order

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


def test_hand_worked_errors_and_order_pin_the_band_width():
    # rho = 1/2 puts the jump at x_c = 0, where c_0 = 1/2, c_1 = -2/pi and
    # c_2 = 0.  Jackson factors: g_1 = 1/2 for m = 1 (alpha = pi/3) and
    # g_1 = 1/sqrt(2) for m = 2 (alpha = pi/4), so p_1(x) = 1/2 - x/pi and
    # p_2(x) = 1/2 - sqrt(2) x/pi.  On the 5-point grid {+-1, +-1/sqrt(2), 0}
    # a band of half-width w = 0.4 lambda_N (|lambda - lambda_c| < 0.4
    # lambda_N, i.e. |x| < 0.8) keeps only x = +-1, where both errors are
    # 1/2 - g_1 (2/pi); had the band been taken as |x| < w it would keep
    # x = +-1/sqrt(2) too, where p_2 errs by 1/2 - 1/pi.
    assert order.band_error(0.5, 1, 0.4, 5) == pytest.approx(0.5 - 1.0 / np.pi, abs=1e-14)
    assert order.band_error(0.5, 2, 0.4, 5) == pytest.approx(0.5 - np.sqrt(2.0) / np.pi, abs=1e-14)
    assert order.m_star(0.5, 0.1, 10, 0.4, 5) == 2
    # with a band that also drops +-1/sqrt(2) only under the wrong width, the
    # two readings part: w = 0.3 keeps |x| >= 0.6, so x = +-1/sqrt(2) counts
    assert order.band_error(0.5, 2, 0.3, 5) == pytest.approx(0.5 - 1.0 / np.pi, abs=1e-14)
    assert order.m_star(0.5, 0.1, 2, 0.3, 5) == 3  # none up to m = 2 meets delta


@pytest.mark.parametrize("rho,w,m,lmax", [(0.17, 0.02, 60, 37.5), (0.05, 0.01, 150, 67.7), (0.5, 0.1, 7, 1.0),
                                          (0.83, 0.03, 25, 12.0)])
def test_band_error_from_the_spectrum_side(rho, w, m, lmax):
    # the same sup written in the spectral variable lambda in [0, lambda_N]:
    # the grid points mapped to lambda = lambda_N (x + 1) / 2, the band taken
    # as |lambda - lambda_c| < w lambda_N with lambda_c = rho lambda_N, the
    # ideal filter as 1[lambda <= lambda_c] and the polynomial evaluated by
    # numpy's Chebyshev series in 2 lambda / lambda_N - 1
    from numpy.polynomial import chebyshev
    lam = lmax * (order.grid_points(G) + 1.0) / 2.0
    lc = rho * lmax
    keep = np.abs(lam - lc) >= w * lmax * (1.0 - 1e-12)
    a = cheb.cheb_coeffs(lc, lmax, m)
    h = (lam[keep] <= lc).astype(np.float64)
    e_lam = float(np.max(np.abs(h - chebyshev.chebval(2.0 * lam[keep] / lmax - 1.0, a))))
    assert order.band_error(rho, m, w, G) == pytest.approx(e_lam, abs=1e-12)
