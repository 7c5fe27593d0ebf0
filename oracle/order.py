"""Choice of the polynomial order m (the note on the choice of m, Sec. 2.4):
m*(lambda_c / lambda_N; delta) is the least order whose approximation of the
ideal low-pass stays within delta of it.  Test infrastructure only.

Reading taken here: the printed criterion takes the sup over all of
[0, lambda_N] of |h - p_m|, which no polynomial meets for delta < 1/2 because
h jumps at lambda_c (and the printed expression mixes the scalar h(lambda)
with a vector).  The sup is therefore taken outside a transition band
|lambda - lambda_c| < w lambda_N, on the fixed grid of G Chebyshev points
x_i = cos(pi i / (G - 1)), i = 0..G-1, of x = 2 lambda / lambda_N - 1:

    E_m(rho) = max_{i : |x_i - x_c| >= 2 w} |h(x_i) - p_m(x_i)|,
    x_c = 2 rho - 1, h(x) = 1[x <= x_c], p_m = sum_{j <= m} a_j T_j,
    m*(rho; delta) = min {m in 1..m_max : E_m(rho) <= delta}  (m_max + 1 if none),

with a_j the Jackson-damped coefficients of the filter (cheb_coeffs).  Here
T_j(x) = cos(j arccos x).

Pinned by (tests/test_oracle_order.py): the mirror symmetry
m*(rho) = m*(1 - rho) (p for 1 - rho is 1 - p(-x) since g_0 = 1, on a grid
symmetric about 0); m* = 1 for delta >= 1 (Jackson-damped step approximations
stay in [0, 1]); monotonicity in delta and in w; the definition itself
(E_{m*} <= delta < E_{m*-1}); the decay of E_m like m^-3 for a fixed band
(the tail of the Jackson kernel), against the stalling of the undamped series;
and the band width itself by hand-worked errors at rho = 1/2 on a 5-point grid
(E_1 = 1/2 - 1/pi, E_2 = 1/2 - sqrt(2)/pi, m*(0.1) = 2 for w = 0.4, where the
band |x - x_c| < w instead would give m* > 2) and by the same sup written in the
spectral variable lambda (band |lambda - lambda_c| < w lambda_N, numpy's
Chebyshev series) at several lambda_N.
"""
from __future__ import annotations

import numpy as np

from .cheb import cheb_coeffs, cheb_eval


def grid_points(G: int) -> np.ndarray:
    return np.cos(np.pi * np.arange(G, dtype=np.float64) / (G - 1))


def band_error(rho: float, m: int, w: float, G: int, jackson: bool = True) -> float:
    """E_m(rho) for band half-width w (fraction of lambda_N); 0 if the band
    covers the whole grid."""
    x = grid_points(G)
    xc = 2.0 * rho - 1.0
    keep = np.abs(x - xc) >= 2.0 * w
    if not np.any(keep):
        return 0.0
    a = cheb_coeffs(rho, 1.0, m, jackson)
    h = (x[keep] <= xc).astype(np.float64)
    return float(np.max(np.abs(h - cheb_eval(a, x[keep]))))


def order_errors(rho: float, m_max: int, w: float, G: int, jackson: bool = True) -> np.ndarray:
    """E_1 .. E_{m_max} (index m - 1)."""
    return np.array([band_error(rho, m, w, G, jackson) for m in range(1, m_max + 1)])


def m_star(rho: float, delta: float, m_max: int, w: float, G: int, jackson: bool = True) -> int:
    for m in range(1, m_max + 1):
        if band_error(rho, m, w, G, jackson) <= delta:
            return m
    return m_max + 1
