"""k-means++ seeding of the k-means step (Sec. 5 runs Matlab's k-means, whose
default start is the D^2 seeding of Arthur and Vassilvitskii, 2007: every new
centre is a data row drawn with probability proportional to its squared
distance to the nearest centre chosen so far).  Test infrastructure only.

Reading taken here, so that the draw is exact and reproducible on any
hardware: the random numbers are 53-bit integers U_c passed in, and the
weights of the draw are the integers
    q_i = floor(2^30 * (D_i / max_j D_j)),
D_i the least squared distance from row i to the rows chosen so far (float64,
columns summed in order, each square rounded before the add).  The first row
is floor(U_0 n / 2^53); row c >= 1 is the least i whose prefix sum
q_0 + ... + q_i exceeds floor(U_c T / 2^53), T = sum_i q_i; if T = 0 (every
row coincides with a chosen one) it is floor(U_c n / 2^53).  All of this is
integer arithmetic except D_i and one division, which IEEE float64 rounds the
same way everywhere.

Pinned by (tests/test_oracle_kmeanspp.py): the D^2 law by the frequency of
the second pick over many draws (against the D law it is not), the integer
mapping at its ends (U = 0, U = 2^53 - 1), a permutation when k = n, the only
distinct row taken second among copies, hand-computed distances.
"""
from __future__ import annotations

import numpy as np

SCALE_BITS = 30
U_BITS = 53


def sqdist_to_row(F: np.ndarray, x: np.ndarray) -> np.ndarray:
    """sum_col (F[:, col] - x[col])^2 in float64, columns in order."""
    d = np.zeros(F.shape[0])
    for col in range(F.shape[1]):
        diff = F[:, col] - x[col]
        sq = diff * diff
        d = d + sq
    return d


def weights(D: np.ndarray) -> np.ndarray:
    """q_i = floor(2^30 (D_i / max D)) as int64 (all zero if max D = 0)."""
    dmax = float(np.max(D))
    if not dmax > 0.0:
        return np.zeros(len(D), dtype=np.int64)
    return np.floor((D / dmax) * float(1 << SCALE_BITS)).astype(np.int64)


def kmeans_pp_rows(F: np.ndarray, k: int, U) -> np.ndarray:
    """Indices (int32, k) of the rows chosen as initial centroids."""
    F = np.asarray(F, dtype=np.float32).astype(np.float64)
    n = F.shape[0]
    U = [int(u) for u in U]
    if not 1 <= k <= n or len(U) < k or any(u < 0 or u >= (1 << U_BITS) for u in U[:k]):
        raise ValueError("need 1 <= k <= n and k integers in [0, 2^53)")
    rows = [(U[0] * n) >> U_BITS]
    D = sqdist_to_row(F, F[rows[0]])
    for c in range(1, k):
        q = weights(D)
        T = int(q.sum())
        if T == 0:
            i = (U[c] * n) >> U_BITS
        else:
            target = (U[c] * T) >> U_BITS
            i = int(np.searchsorted(np.cumsum(q), target, side="right"))
        rows.append(i)
        D = np.minimum(D, sqdist_to_row(F, F[i]))
    return np.asarray(rows, dtype=np.int32)

