"""Pins of the oracle's polynomial low-pass filter (Eq. ideal, Sec. 2.3-2.4, Sec. 3.1)."""
import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads as W


def _L(g):
    return oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, g.w)


@pytest.mark.parametrize("xc", [-0.9, -0.31, 0.0, 0.42, 0.97])
def test_step_coeffs_vs_integration(xc):
    # Chebyshev projection c_j = (2/pi) int_0^pi h(cos t) cos(j t) dt (c_0 with 1/pi),
    # integrated numerically on [theta, pi] where h = 1
    lmax = 7.0
    lc = (xc + 1) * lmax / 2
    p = 40
    c = oracle.step_coeffs(lc, lmax, p)
    th = np.arccos(xc)
    for j in range(p + 1):
        val, _ = integrate.quad(lambda t: np.cos(j * t), th, np.pi, epsabs=1e-13, epsrel=1e-12, limit=200)
        ref = val / np.pi if j == 0 else 2 * val / np.pi
        assert abs(c[j] - ref) < 1e-12, j


@pytest.mark.parametrize("p", [1, 2, 7, 50, 150])
def test_jackson_is_sine_window_autocorrelation(p):
    # Jackson damping = normalised autocorrelation of the window sin(pi (k+1)/(p+2)), k = 0..p
    v = np.sin(np.pi * (np.arange(p + 1) + 1) / (p + 2))
    ac = np.array([np.dot(v[: p + 1 - j], v[j:]) for j in range(p + 1)]) / np.dot(v, v)
    np.testing.assert_allclose(oracle.jackson(p), ac, atol=1e-14)
    assert oracle.jackson(p)[0] == pytest.approx(1.0, abs=1e-15)


def test_special_cases():
    p = 30
    # all-pass: cut-off at or above lambda_max -> p(x) = 1 -> a = (1, 0, ..., 0)
    for lc in (5.0, 6.0):
        a = oracle.cheb_coeffs(lc, 5.0, p)
        assert a[0] == pytest.approx(1.0, abs=1e-15)
        np.testing.assert_allclose(a[1:], 0, atol=1e-15)
    # all-stop below 0: x_c = -1 -> theta = pi -> a = 0
    np.testing.assert_allclose(oracle.cheb_coeffs(-1.0, 5.0, p), 0, atol=1e-15)
    # half band: x_c = 0 -> c_0 = 1/2, even c_j = 0
    c = oracle.step_coeffs(2.5, 5.0, p)
    assert c[0] == pytest.approx(0.5, abs=1e-15)
    np.testing.assert_allclose(c[2::2], 0, atol=1e-15)


@pytest.mark.parametrize("p", [10, 50, 100, 150, 200])
@pytest.mark.parametrize("frac", [1e-4, 0.05, 0.17, 0.5, 0.9])
def test_jackson_positivity(p, frac):
    # convolution of the step with a positive kernel of unit mass: 0 <= p(x) <= 1
    a = oracle.cheb_coeffs(frac, 1.0, p)
    x = np.linspace(-1, 1, 4001)
    px = oracle.cheb_eval(a, x)
    assert px.min() >= -1e-12 and px.max() <= 1 + 1e-12
    # without damping the Gibbs overshoot is visible
    if p >= 50 and 0.05 <= frac <= 0.9:
        assert oracle.cheb_eval(oracle.cheb_coeffs(frac, 1.0, p, False), x).max() > 1.05


def test_cheb_eval_vs_recurrence():
    a = np.random.default_rng(0).standard_normal(20)
    x = np.linspace(-1, 1, 101)
    t_prev, t = np.ones_like(x), x.copy()
    ref = a[0] * t_prev + a[1] * t
    for j in range(2, 20):
        t_prev, t = t, 2 * x * t - t_prev
        ref += a[j] * t
    np.testing.assert_allclose(oracle.cheb_eval(a, x), ref, atol=1e-12)


@pytest.mark.parametrize("make", [lambda: W.random_weighted(50, 0.2, 1), lambda: W.workload_graph(1),
                                  lambda: W.cliques(4, 6, True), lambda: W.random_weighted(30, 0.2, 5, isolated=4)])
@pytest.mark.parametrize("p", [0, 1, 2, 17, 50])
def test_recurrence_equals_dense_matrix_polynomial(make, p):
    g = make()
    L = _L(g)
    lam, chi = oracle.dense_spectrum(L.toarray())
    lmax = lam[-1] * 1.01
    R, _ = W.signals(g.n, 8, 3)
    R = R.astype(np.float64)
    a = oracle.cheb_coeffs(0.3 * lmax, lmax, p)
    Y = oracle.cheb_filter(L, lmax, a, R)
    Yd = oracle.dense_filter(lam, chi, lmax, a, R)
    assert np.linalg.norm(Y - Yd) <= 1e-10 * max(np.linalg.norm(Yd), 1e-300) + 1e-13


def test_spectral_error_identity():
    # |Y - H R|_F^2 = sum_l (p(x_l) - h(lambda_l))^2 |chi_l^T R|^2 (exact, Sec. 3.1 projector)
    g = W.workload_graph(1)
    L = _L(g)
    lam, chi = oracle.dense_spectrum(L.toarray())
    lmax = lam[-1] * 1.01
    k = 10
    lc = 0.5 * (lam[k - 1] + lam[k])
    R = W.signals(g.n, 32, 7)[1]
    a = oracle.cheb_coeffs(lc, lmax, 50)
    Y = oracle.cheb_filter(L, lmax, a, R)
    H = oracle.ideal_filter(lam, chi, lc, R)
    px = oracle.cheb_eval(a, 2 * lam / lmax - 1)
    h = (lam <= lc).astype(float)
    rhat2 = np.sum((chi.T @ R) ** 2, axis=1)
    lhs = np.sum((Y - H) ** 2)
    rhs = np.sum((px - h) ** 2 * rhat2)
    assert lhs == pytest.approx(rhs, rel=1e-9)
    # with cut-off between lambda_k and lambda_{k+1} the ideal filter is U U^T
    U = chi[:, :k]
    np.testing.assert_allclose(H, U @ (U.T @ R), atol=1e-12)


def test_disjoint_cliques_projector():
    # k disjoint cliques: eigenvalue 0 has the k block indicators as eigenvectors,
    # so the ideal filter at any cut-off in [0, m) is the block-averaging projector
    k, m = 4, 5
    g = W.cliques(k, m)
    L = _L(g)
    lam, chi = oracle.dense_spectrum(L.toarray())
    R = W.signals(g.n, 6, 2)[1]
    H = oracle.ideal_filter(lam, chi, 1.0, R)
    ref = np.repeat(R.reshape(k, m, -1).mean(axis=1), m, axis=0)
    np.testing.assert_allclose(H, ref, atol=1e-12)
    # a high-order damped polynomial approaches it (eigengap m)
    lmax = m * 1.01
    Y = oracle.cheb_filter(L, lmax, oracle.cheb_coeffs(0.5 * m, lmax, 200), R)
    assert np.linalg.norm(Y - ref) < 2e-2 * np.linalg.norm(ref)


@pytest.mark.parametrize("p", [50, 100, 150])
def test_constant_vector_gain(p):
    # L 1 = 0 -> x = -1 -> Y(1) = p(-1) 1, p(-1) = sum_j a_j (-1)^j (close to 1)
    g = W.workload_graph(1)
    L = _L(g)
    lmax = 40.0
    a = oracle.cheb_coeffs(0.17 * lmax, lmax, p)
    Y = oracle.cheb_filter(L, lmax, a, np.ones((g.n, 1)))
    pm1 = float(np.sum(a * (-1.0) ** np.arange(p + 1)))
    np.testing.assert_allclose(Y[:, 0], pm1, rtol=1e-12)
    assert 0.99 < pm1 <= 1.0


@pytest.mark.parametrize("n", [6, 9])
def test_closed_form_complete_graph_filter(n):
    # K_n: L = n I - 1 1^T; a low-pass below n keeps only the mean
    g = W.complete(n)
    L = _L(g)
    lmax = n * 1.05
    R = W.signals(n, 4, 1)[1]
    a = oracle.cheb_coeffs(0.5 * n, lmax, 30)
    Y = oracle.cheb_filter(L, lmax, a, R)
    p0 = oracle.cheb_eval(a, -1.0)
    pn = oracle.cheb_eval(a, 2 * n / lmax - 1)
    mean = R.mean(axis=0, keepdims=True)
    ref = p0 * np.repeat(mean, n, 0) + pn * (R - mean)
    np.testing.assert_allclose(Y, ref, atol=1e-12)
