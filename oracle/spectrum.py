"""Spectrum of L and the estimate of its largest eigenvalue (Sec. 2.1; step 1
of the algorithm in Sec. 4.1).  Test infrastructure only.

The paper only says that lambda_N is *estimated*, citing a numerical linear
algebra textbook.  Reading taken here: the Lanczos iteration in float64 from a
given start vector, without re-orthogonalisation, for a fixed number of
iterations (stopping early on breakdown), whose largest Ritz value is a lower
bound of lambda_N; the estimate is that Ritz value times 1.01, clipped to the
Gershgorin bound 2 max_i s_i (every eigenvalue of L = S - W lies in
[0, 2 max s_i]).

Pinned by: dense eigh on tiny graphs and closed-form spectra (complete graph,
cycle, path), the bounds max_i s_i <= lambda_N <= 2 max_i s_i
(tests/test_oracle_spectrum.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# breakdown threshold of the Lanczos iteration, relative to max_i s_i
LANCZOS_BREAKDOWN = 1e-12
LMAX_MARGIN = 1.01


def dense_spectrum(L: np.ndarray):
    """(lambda ascending, chi orthonormal eigenvectors) of a dense symmetric L."""
    lam, chi = np.linalg.eigh(np.asarray(L, dtype=np.float64))
    return lam, chi


def lambda_max_exact(L) -> float:
    if sp.issparse(L):
        if L.shape[0] <= 3000:
            return float(np.linalg.eigvalsh(L.toarray())[-1])
        from scipy.sparse.linalg import eigsh
        return float(eigsh(L, k=1, which="LA", tol=1e-12, return_eigenvectors=False)[0])
    return float(np.linalg.eigvalsh(L)[-1])


def lanczos_tridiag(L, v0: np.ndarray, iters: int, smax: float):
    """Plain Lanczos: returns (alpha[m], beta[m-1]) of the m x m tridiagonal.

    v_1 = v0/|v0|; w = L v_j - beta_j v_{j-1}; alpha_j = <w, v_j>;
    w -= alpha_j v_j; beta_{j+1} = |w|; v_{j+1} = w / beta_{j+1}.
    Stops after ``iters`` steps or when beta_{j+1} <= 1e-12 max_i s_i.
    """
    v = np.asarray(v0, dtype=np.float64) / np.linalg.norm(v0)
    v_prev = np.zeros_like(v)
    beta = 0.0
    alphas, betas = [], []
    for j in range(iters):
        w = L @ v - beta * v_prev
        a = float(np.dot(w, v))
        w = w - a * v
        alphas.append(a)
        beta = float(np.linalg.norm(w))
        if j == iters - 1 or beta <= LANCZOS_BREAKDOWN * smax:
            break
        betas.append(beta)
        v_prev = v
        v = w / beta
    return np.array(alphas), np.array(betas)


def lanczos_lmax(L, v0, iters, smax):
    """Largest Ritz value of the Lanczos tridiagonal (a lower bound of lambda_N)."""
    a, b = lanczos_tridiag(L, v0, iters, smax)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    return float(np.linalg.eigvalsh(T)[-1])


def lmax_estimate(L, s: np.ndarray, v0, iters: int = 60) -> float:
    """min(1.01 * largest Ritz value, 2 max_i s_i)."""
    smax = float(np.max(s)) if len(s) else 0.0
    theta = lanczos_lmax(L, v0, iters, smax)
    return float(min(LMAX_MARGIN * theta, 2.0 * smax))
