"""Estimate of the number of eigenvalues below a cut-off and the dichotomy that
estimates lambda_k (Sec. 3.2; step 2 of the algorithm in Sec. 4.1).  Test
infrastructure only.

The paper counts eigenvalues below lambda_c by filtering random signals (after
the spectral-density method it cites) and bisects on [0, lambda_N].  Reading
taken here:

  count(lambda_c) = <R, p_{lambda_c}(L~) R>_F
                  = sum_j a_j(lambda_c) mu_j,   mu_j = <R, T_j(L~) R>_F,

an unbiased estimate of tr p(L~) = sum_l p(x_l) ~ #{l : lambda_l <= lambda_c}
when the entries of R are i.i.d. with variance 1/R.  Dichotomy: lo = 0,
hi = lambda_max; for S steps mid = (lo+hi)/2, hi = mid if count(mid) >= k - 1/2
else lo = mid; the estimate is hi.

Pinned by (tests/test_oracle_eigcount.py): with R = I_N the count equals
sum_l p(x_l) from the dense spectrum; the Hutchinson mean over seeds matches the
trace within 3 standard errors; on graphs with a large k-th eigengap the
rounded count equals the exact count and the dichotomy lands inside
(lambda_k, lambda_{k+1}); the moment route equals the literal route <R, Y>.
"""
from __future__ import annotations

import numpy as np

from .cheb import cheb_coeffs, cheb_filter, cheb_states


def moments(L, lmax: float, p: int, R: np.ndarray) -> np.ndarray:
    """mu_j = <R, T_j(L~) R>_F, j = 0..p (float64)."""
    R = np.asarray(R, dtype=np.float64)
    return np.array([float(np.sum(R * t)) for t in cheb_states(L, lmax, p, R)])


def eigcount_from_moments(mu: np.ndarray, lambda_c: float, lmax: float, use_jackson: bool = True) -> float:
    p = len(mu) - 1
    return float(np.dot(cheb_coeffs(lambda_c, lmax, p, use_jackson), mu))


def eigcount_literal(L, lmax: float, lambda_c: float, p: int, R: np.ndarray, use_jackson: bool = True) -> float:
    """<R, Y> with Y the filtered signals at cut-off lambda_c."""
    a = cheb_coeffs(lambda_c, lmax, p, use_jackson)
    return float(np.sum(np.asarray(R, dtype=np.float64) * cheb_filter(L, lmax, a, R)))


def exact_count(lam: np.ndarray, lambda_c: float) -> int:
    return int(np.sum(lam <= lambda_c))


def dichotomy(count_fn, lmax: float, k: int, steps: int):
    """Bisection on [0, lambda_max] for the smallest cut-off whose count reaches k.
    Returns (estimate, trajectory [(mid, count)])."""
    lo, hi = 0.0, float(lmax)
    traj = []
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        c = count_fn(mid)
        traj.append((mid, c))
        if c >= k - 0.5:
            hi = mid
        else:
            lo = mid
    return hi, np.array(traj).reshape(-1, 2)


def dichotomy_moments(L, lmax, k, p, steps, R, use_jackson=True):
    mu = moments(L, lmax, p, R)
    return dichotomy(lambda lc: eigcount_from_moments(mu, lc, lmax, use_jackson), lmax, k, steps)


def dichotomy_literal(L, lmax, k, p, steps, R, use_jackson=True):
    return dichotomy(lambda lc: eigcount_literal(L, lmax, lc, p, R, use_jackson), lmax, k, steps)
