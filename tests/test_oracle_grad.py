"""Pins of the oracle's gradients (adjoint of the recurrence; extension of Sec. 2.4)."""
import numpy as np
import pytest

import oracle
import workloads as W


def _setup(seed=1, n=14, p=9, r=3):
    g = W.random_weighted(n, 0.4, seed)
    w = g.w.astype(np.float64)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, w)
    lam, chi = oracle.dense_spectrum(L.toarray())
    lmax = lam[-1] * 1.02
    a = oracle.cheb_coeffs(0.35 * lmax, lmax, p)
    R = W.signals_f64(g.n, r, seed + 10)
    T = W.unit_rows(g.n, r, seed + 20).astype(np.float64)
    return g, w, L, lam, chi, lmax, a, R, T


@pytest.mark.parametrize("p", [1, 2, 3, 9])
def test_adjoint_vs_finite_differences(p):
    g, w, L, lam, chi, lmax, a, R, T = _setup(p=p)
    a = oracle.cheb_coeffs(0.35 * lmax, lmax, p)
    Y = oracle.cheb_filter(L, lmax, a, R)
    loss, G = oracle.rownorm_loss_grad(Y, T)
    dw, da = oracle.cheb_filter_adjoint(g.n, g.row_ptr, g.col_idx, w, lmax, a, R, G)
    h = 1e-6
    for e in range(g.nnz):
        wp, wm = w.copy(), w.copy()
        wp[e] += h
        wm[e] -= h
        fd = (oracle.loss_of_weights(g.n, g.row_ptr, g.col_idx, wp, lmax, a, R, T)
              - oracle.loss_of_weights(g.n, g.row_ptr, g.col_idx, wm, lmax, a, R, T)) / (2 * h)
        assert dw[e] == pytest.approx(fd, rel=1e-6, abs=1e-8), e
    # coefficient gradient: the loss depends on a through Y = sum_j a_j T_j R
    for j in range(p + 1):
        ap, am = a.copy(), a.copy()
        ap[j] += h
        am[j] -= h
        fd = (oracle.rownorm_loss_grad(oracle.cheb_filter(L, lmax, ap, R), T)[0]
              - oracle.rownorm_loss_grad(oracle.cheb_filter(L, lmax, am, R), T)[0]) / (2 * h)
        assert da[j] == pytest.approx(fd, rel=1e-6, abs=1e-8), j


def test_adjoint_vs_daleckii_krein():
    g, w, L, lam, chi, lmax, a, R, T = _setup(seed=3, n=18, p=25, r=4)
    G = W.signals_f64(g.n, 4, 77)  # any cotangent
    dw, _ = oracle.cheb_filter_adjoint(g.n, g.row_ptr, g.col_idx, w, lmax, a, R, G)
    M = oracle.daleckii_krein_M(lam, chi, lmax, a, R, G)
    dw_dk = oracle.dW_from_M(M, g.n, g.row_ptr, g.col_idx, lmax)
    np.testing.assert_allclose(dw, dw_dk, rtol=1e-7, atol=1e-10 * np.abs(dw_dk).max())


def test_dsigma_vs_finite_differences():
    g = W.gmm_knn(300, 4, 3, 5, 7)
    sigma = 2.0
    d2 = g.d2.astype(np.float64)
    w = oracle.gauss_weights(d2, sigma)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, w)
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, w)
    lmax = oracle.lmax_estimate(L, s, W.start_vector(g.n, 1), 80)
    a = oracle.cheb_coeffs(0.1 * lmax, lmax, 12)
    R = W.signals_f64(g.n, 4, 5)
    T = W.unit_rows(g.n, 4, 6).astype(np.float64)
    Y = oracle.cheb_filter(L, lmax, a, R)
    _, G = oracle.rownorm_loss_grad(Y, T)
    dw, _ = oracle.cheb_filter_adjoint(g.n, g.row_ptr, g.col_idx, w, lmax, a, R, G)
    ds = oracle.dsigma(dw, w, d2, sigma)
    h = 1e-6
    fp = oracle.loss_of_weights(g.n, g.row_ptr, g.col_idx, oracle.gauss_weights(d2, sigma + h), lmax, a, R, T)
    fm = oracle.loss_of_weights(g.n, g.row_ptr, g.col_idx, oracle.gauss_weights(d2, sigma - h), lmax, a, R, T)
    assert ds == pytest.approx((fp - fm) / (2 * h), rel=1e-6)


def test_loss_grad_vs_finite_differences():
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((6, 4))
    T = W.unit_rows(6, 4, 3)
    loss, G = oracle.rownorm_loss_grad(Y, T)
    h = 1e-7
    for i in range(6):
        for r in range(4):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[i, r] += h
            Ym[i, r] -= h
            fd = (oracle.rownorm_loss_grad(Yp, T)[0] - oracle.rownorm_loss_grad(Ym, T)[0]) / (2 * h)
            assert G[i, r] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_sampled_adjoint_equals_full():
    g, w, L, lam, chi, lmax, a, R, T = _setup(seed=4, n=30, p=12, r=3)
    G = W.signals_f64(g.n, 3, 8)
    dw, da = oracle.cheb_filter_adjoint(g.n, g.row_ptr, g.col_idx, w, lmax, a, R, G)
    ent = np.array([0, 3, g.nnz - 1, g.nnz // 2])
    dws, das = oracle.cheb_filter_adjoint_sampled(g.n, g.row_ptr, g.col_idx, w, lmax, a, R, G, ent)
    np.testing.assert_allclose(dws, dw[ent], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(das, da, rtol=1e-13)


def test_adjoint_term_scale_bounds_the_gradient():
    # the optional scale (sum over the steps of the two terms' absolute
    # values) bounds |dw| entrywise by the triangle inequality, and asking
    # for it leaves dw and da as they are
    g = W.random_weighted(60, 0.15, 8, isolated=2)
    w = g.w.astype(np.float64)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, w)
    lmax = 1.01 * oracle.lambda_max_exact(L)
    a = oracle.cheb_coeffs(0.3 * lmax, lmax, 25)
    _, R = W.signals(g.n, 4, 1)
    G = W.signals_f64(g.n, 4, 2)
    dw, da = oracle.cheb_filter_adjoint(g.n, g.row_ptr, g.col_idx, w, lmax, a, R, G)
    dw2, da2, scale = oracle.cheb_filter_adjoint(g.n, g.row_ptr, g.col_idx, w, lmax, a, R, G, with_scale=True)
    np.testing.assert_array_equal(dw, dw2)
    np.testing.assert_array_equal(da, da2)
    assert np.all(np.abs(dw) <= scale * (1 + 1e-12))
    assert np.all(scale > 0)
    z, _, zs = oracle.cheb_filter_adjoint(g.n, g.row_ptr, g.col_idx, w, lmax, a[:1], R, G, with_scale=True)
    assert not np.any(z) and not np.any(zs)
