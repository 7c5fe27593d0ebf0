"""Ideal low-pass filter and its polynomial approximation (Eq. ideal, Sec. 2.3,
Sec. 2.4, Sec. 3.1, steps 3-5 of the algorithm in Sec. 4.1).  Test
infrastructure only.

The paper writes the fast filter as an order-m polynomial of L applied to the
signals.  Reading taken here (the monomial basis being unusable at m ~ 100):
the polynomial is expanded in Chebyshev polynomials of the spectrum mapped to
[-1, 1] by x = 2 lambda / lambda_max - 1, i.e. of L~ = (2/lambda_max) L - I,

    p(x) = sum_{j=0..p} a_j T_j(x),   a_j = g_j c_j,

with c_j the exact Chebyshev coefficients of the step 1[x <= x_c] (full c_0,
not halved) and g_j the Jackson damping factors.  The filter of a block R is
evaluated by the three-term recurrence T_0 = R, T_1 = L~ R,
T_{j+1} = 2 L~ T_j - T_{j-1}, Y = sum_j a_j T_j.

Pinned by (tests/test_oracle_cheb.py): coefficients against numerical
integration of the Chebyshev projection; the Jackson factors against the
normalised autocorrelation of a sine window; the all-pass and half-band special
cases; 0 <= p(x) <= 1; recurrence against the dense matrix function
chi diag(p(x_l)) chi^T; the exact spectral-error identity against the ideal
projector of Sec. 3.1; closed-form spectra; the constant-vector gain.
"""
from __future__ import annotations

import numpy as np


def jackson(p: int) -> np.ndarray:
    """Jackson damping g_0..g_p for an order-p expansion (p+1 terms):
    g_j = [(p+2-j) cos(j a) + sin(j a) cot(a)] / (p+2), a = pi/(p+2)."""
    j = np.arange(p + 1, dtype=np.float64)
    a = np.pi / (p + 2)
    return ((p + 2 - j) * np.cos(j * a) + np.sin(j * a) / np.tan(a)) / (p + 2)


def step_coeffs(lambda_c: float, lmax: float, p: int) -> np.ndarray:
    """Chebyshev coefficients c_0..c_p of h(x) = 1[x <= x_c] on [-1, 1],
    x_c = clip(2 lambda_c / lambda_max - 1, -1, 1), theta = arccos x_c:
    c_0 = 1 - theta/pi, c_j = -2 sin(j theta)/(j pi)."""
    xc = min(max(2.0 * lambda_c / lmax - 1.0, -1.0), 1.0)
    th = np.arccos(xc)
    c = np.empty(p + 1)
    c[0] = 1.0 - th / np.pi
    j = np.arange(1, p + 1, dtype=np.float64)
    c[1:] = -2.0 * np.sin(j * th) / (j * np.pi)
    return c


def cheb_coeffs(lambda_c: float, lmax: float, p: int, use_jackson: bool = True) -> np.ndarray:
    """a_j = g_j c_j (g = 1 without damping)."""
    c = step_coeffs(lambda_c, lmax, p)
    return c * jackson(p) if use_jackson else c


def cheb_eval(a: np.ndarray, x) -> np.ndarray:
    """p(x) = sum_j a_j T_j(x) with T_j(x) = cos(j arccos x) on [-1, 1]."""
    x = np.clip(np.asarray(x, dtype=np.float64), -1.0, 1.0)
    t = np.arccos(x)
    j = np.arange(len(a), dtype=np.float64)
    return np.cos(np.multiply.outer(t, j)) @ np.asarray(a, dtype=np.float64)


def scaled_laplacian(L, lmax: float):
    """L~ = (2/lambda_max) L - I (sparse or dense)."""
    import scipy.sparse as sp
    n = L.shape[0]
    if sp.issparse(L):
        return ((2.0 / lmax) * L - sp.identity(n)).tocsr()
    return (2.0 / lmax) * L - np.eye(n)


def cheb_states(L, lmax: float, p: int, R: np.ndarray):
    """Yields T_0 R, ..., T_p R (float64) by the three-term recurrence."""
    Lt = scaled_laplacian(L, lmax)
    R = np.asarray(R, dtype=np.float64)
    t_prev = R
    yield t_prev
    if p == 0:
        return
    t = Lt @ R
    yield t
    for _ in range(1, p):
        t_next = 2.0 * (Lt @ t) - t_prev
        t_prev, t = t, t_next
        yield t


def cheb_filter(L, lmax: float, a: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Y = sum_{j=0..p} a_j T_j(L~) R, p = len(a) - 1 (the fast filter of Sec. 2.4)."""
    p = len(a) - 1
    Y = np.zeros(np.shape(R), dtype=np.float64)
    for j, t in enumerate(cheb_states(L, lmax, p, R)):
        Y += a[j] * t
    return Y


def dense_filter(lam: np.ndarray, chi: np.ndarray, lmax: float, a: np.ndarray, R: np.ndarray) -> np.ndarray:
    """chi diag(p(x_l)) chi^T R with x_l = 2 lambda_l / lambda_max - 1 (graph filter
    operator of Sec. 2.3 with h replaced by the polynomial)."""
    px = cheb_eval(a, 2.0 * lam / lmax - 1.0)
    return chi @ (px[:, None] * (chi.T @ R))


def ideal_filter(lam: np.ndarray, chi: np.ndarray, lambda_c: float, R: np.ndarray) -> np.ndarray:
    """H_{lambda_c} R = chi diag(1[lambda_l <= lambda_c]) chi^T R (Eq. ideal);
    equals U U^T R when lambda_c = lambda_k < lambda_{k+1} (Sec. 3.1)."""
    h = (lam <= lambda_c).astype(np.float64)
    return chi @ (h[:, None] * (chi.T @ R))
