"""Gradients of a loss on the filtered features with respect to the edge
weights, the Gaussian-kernel bandwidth and the filter coefficients.  Test
infrastructure only.

This goes beyond the paper (which has no differentiation); the similarity
graph is the Gaussian kernel of Sec. 2.2 step 1, w_e = exp(-d_e^2 / sigma^2).
Conventions (readings):
  * lambda_max is a constant (not differentiated);
  * every *stored* CSR entry e = (i, k) is its own parameter: it enters the
    operator as applied by row i, i.e. L_ik = -w_e and L_ii = sum_e w_e, so
    dL~/dw_e = (2/lambda_max)(E_ii - E_ik); the gradient of an undirected edge
    is the sum of its two stored entries;
  * loss = sum_i |f_hat_i - t_i|^2 with f_hat_i = y_i/|y_i| (a sum, not a mean).

Adjoint of the recurrence (reverse mode written out):
  A_p = a_p G,  A_{p-1} = a_{p-1} G + 2 L~ A_p,
  A_j = a_j G + 2 L~ A_{j+1} - A_{j+2}   (1 <= j <= p-2),
  M = dloss/dL~ = A_1 T_0^T + sum_{j=1..p-1} 2 A_{j+1} T_j^T,
  dw_e = (2/lambda_max)(M_ii - M_ik),  da_j = <G, T_j R>,
  dsigma = sum_e dw_e w_e 2 d_e^2 / sigma^3.

Pinned by (tests/test_oracle_grad.py): central finite differences of the loss
through the float64 recurrence; the Daleckii-Krein (divided-difference)
formula for the Frechet derivative of the matrix function on tiny graphs;
linearity of the loss gradient in a.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .cheb import cheb_eval, cheb_filter, cheb_states, scaled_laplacian
from .cluster import normalize_rows


def gauss_weights(d2: np.ndarray, sigma: float) -> np.ndarray:
    return np.exp(-np.asarray(d2, dtype=np.float64) / (sigma * sigma))


def rownorm_loss_grad(Y: np.ndarray, T: np.ndarray):
    """(loss, G = dloss/dY) for loss = sum_i |y_i/|y_i| - t_i|^2.
    G_i = (g_i - f_i (f_i . g_i)) / |y_i| with g_i = 2 (f_i - t_i); zero rows get G_i = 0."""
    F, nrm = normalize_rows(Y)
    T = np.asarray(T, dtype=np.float64)
    diff = F - T
    loss = float(np.sum(diff * diff))
    g = 2.0 * diff
    G = np.zeros_like(F)
    nz = nrm > 0
    proj = np.sum(F * g, axis=1)
    G[nz] = (g[nz] - F[nz] * proj[nz, None]) / nrm[nz, None]
    return loss, G


def _operator(n, row_ptr, col_idx, w):
    """L = S - W built row-wise from the stored entries (need not be symmetric)."""
    W = sp.csr_matrix((np.asarray(w, dtype=np.float64), col_idx, row_ptr), shape=(n, n))
    s = np.asarray(W.sum(axis=1)).reshape(-1)
    return (sp.diags(s) - W).tocsr()


def cheb_filter_adjoint(n, row_ptr, col_idx, w, lmax, a, R, G, with_scale=False):
    """(dw per stored entry, da) of <G, Y> with Y = sum_j a_j T_j(L~) R.

    with_scale: also the per-entry sum over the steps of the absolute values of
    the two terms each step adds to dw, (2/lmax) sum_j (|diag term| + |entry
    term|), the scale on which rounding of those terms acts (dw itself can be
    far smaller when they cancel)."""
    a = np.asarray(a, dtype=np.float64)
    p = len(a) - 1
    L = _operator(n, row_ptr, col_idx, w)
    Lt = scaled_laplacian(L, lmax)
    LtT = Lt.T.tocsr()
    G = np.asarray(G, dtype=np.float64)
    T = list(cheb_states(L, lmax, p, R))
    da = np.array([float(np.sum(G * t)) for t in T])
    rows = np.repeat(np.arange(n), np.diff(np.asarray(row_ptr, dtype=np.int64)))
    cols = np.asarray(col_idx, dtype=np.int64)
    if p == 0:
        z = np.zeros(len(cols))
        return (z, da, z.copy()) if with_scale else (z, da)
    # adjoints A_j for j = 1..p (A[j])
    A = [None] * (p + 2)
    A[p + 1] = np.zeros_like(G)
    A[p] = a[p] * G
    for j in range(p - 1, 0, -1):
        nxt2 = A[j + 2] if j + 2 <= p else 0.0
        A[j] = a[j] * G + 2.0 * (LtT @ A[j + 1]) - nxt2
    # M restricted to the stored pattern and the diagonal
    m_off = np.zeros(len(cols))
    m_diag = np.zeros(n)
    absum = np.zeros(len(cols)) if with_scale else None
    for j in range(0, p):
        cj = 1.0 if j == 0 else 2.0
        Aj1 = A[j + 1]
        Tj = T[j]
        t_off = cj * np.sum(Aj1[rows] * Tj[cols], axis=1)
        t_diag = cj * np.sum(Aj1 * Tj, axis=1)
        m_off += t_off
        m_diag += t_diag
        if with_scale:
            absum += np.abs(t_diag)[rows] + np.abs(t_off)
    dw = (2.0 / lmax) * (m_diag[rows] - m_off)
    if with_scale:
        return dw, da, (2.0 / lmax) * absum
    return dw, da


def daleckii_krein_M(lam, chi, lmax, a, R, G):
    """dloss/dL~ for loss = <G, p(L~) R> via the divided differences of p:
    M = chi (Gamma o (chi^T G R^T chi)) chi^T, Gamma_ab = (p(x_a)-p(x_b))/(x_a-x_b),
    p'(x_a) on the diagonal (and where |x_a - x_b| < 1e-9)."""
    a = np.asarray(a, dtype=np.float64)
    x = 2.0 * lam / lmax - 1.0
    px = cheb_eval(a, x)
    # p'(x) = sum_j a_j j U_{j-1}(x), U by its three-term recurrence
    dp = np.zeros_like(x)
    u_prev, u = np.zeros_like(x), np.ones_like(x)   # U_{-1}, U_0
    for j in range(1, len(a)):
        dp += a[j] * j * u
        u_prev, u = u, 2.0 * x * u - u_prev
    dx = x[:, None] - x[None, :]
    close = np.abs(dx) < 1e-9
    Gam = np.where(close, 0.5 * (dp[:, None] + dp[None, :]),
                   (px[:, None] - px[None, :]) / np.where(close, 1.0, dx))
    inner = chi.T @ np.asarray(G, dtype=np.float64) @ np.asarray(R, dtype=np.float64).T @ chi
    return chi @ (Gam * inner) @ chi.T


def dW_from_M(M, n, row_ptr, col_idx, lmax):
    rows = np.repeat(np.arange(n), np.diff(np.asarray(row_ptr, dtype=np.int64)))
    cols = np.asarray(col_idx, dtype=np.int64)
    return (2.0 / lmax) * (M[rows, rows] - M[rows, cols])


def dsigma(dw, w, d2, sigma) -> float:
    return float(np.sum(np.asarray(dw) * np.asarray(w) * 2.0 * np.asarray(d2, dtype=np.float64) / sigma ** 3))


def loss_of_weights(n, row_ptr, col_idx, w, lmax, a, R, T):
    """loss(rownorm(Y(w))) through the float64 recurrence (for finite differences)."""
    L = _operator(n, row_ptr, col_idx, w)
    Y = cheb_filter(L, lmax, a, R)
    return rownorm_loss_grad(Y, T)[0]


def cheb_filter_adjoint_sampled(n, row_ptr, col_idx, w, lmax, a, R, G, entries):
    """Like cheb_filter_adjoint, but dw only for the stored entries `entries`
    (indices into col_idx): the recurrences run at full size while only the
    rows that the sampled M_ii and M_ik need are kept, so large graphs fit.
    Returns (dw[entries], da)."""
    a = np.asarray(a, dtype=np.float64)
    p = len(a) - 1
    entries = np.asarray(entries, dtype=np.int64)
    rows_all = np.repeat(np.arange(n), np.diff(np.asarray(row_ptr, dtype=np.int64)))
    ri = rows_all[entries]
    ck = np.asarray(col_idx, dtype=np.int64)[entries]
    L = _operator(n, row_ptr, col_idx, w)
    Lt = scaled_laplacian(L, lmax)
    LtT = Lt.T.tocsr()
    G = np.asarray(G, dtype=np.float64)
    T_i, T_k, da = [], [], []
    for t in cheb_states(L, lmax, p, R):
        T_i.append(t[ri].copy())
        T_k.append(t[ck].copy())
        da.append(float(np.sum(G * t)))
    if p == 0:
        return np.zeros(len(entries)), np.array(da)
    m_off = np.zeros(len(entries))
    m_diag = np.zeros(len(entries))
    A_next2 = np.zeros_like(G)       # A_{j+2}
    A_next = a[p] * G                # A_{j+1}, starting at A_p
    for j in range(p - 1, -1, -1):
        cj = 1.0 if j == 0 else 2.0
        m_off += cj * np.sum(A_next[ri] * T_k[j], axis=1)
        m_diag += cj * np.sum(A_next[ri] * T_i[j], axis=1)
        if j >= 1:
            A_j = a[j] * G + 2.0 * (LtT @ A_next) - A_next2
            A_next2, A_next = A_next, A_j
    return (2.0 / lmax) * (m_diag - m_off), np.array(da)
