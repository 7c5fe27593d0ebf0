"""Row normalisation and k-means on the filtered features (step 4 of Sec. 2.2,
step 6 of the algorithm in Sec. 4.1; normalisation after the normalised-
Laplacian footnote of Sec. 2.1).  Test infrastructure only.

Readings taken here: rows of zero norm stay zero; k-means is Lloyd's iteration
from caller-given initial centroids for a fixed number of iterations, the
squared Euclidean distance accumulated in float64 over the columns in order,
ties resolved to the lowest centroid index, and an empty cluster keeps its
previous centroid.

Pinned by (tests/test_oracle_cluster.py): unit row norms and zero rows; a
pure-Python brute-force assignment on tiny inputs, explicit ties; the mean of
members against a per-cluster loop; recovery of disjoint cliques from their
exact ideal-filter features.
"""
from __future__ import annotations

import numpy as np


def normalize_rows(Y: np.ndarray):
    """(f_hat, norms): f_hat_i = y_i / |y_i| if |y_i| > 0 else 0."""
    Y = np.asarray(Y, dtype=np.float64)
    nrm = np.sqrt(np.sum(Y * Y, axis=1))
    out = np.zeros_like(Y)
    nz = nrm > 0
    out[nz] = Y[nz] / nrm[nz, None]
    return out, nrm


def kmeans_assign(F: np.ndarray, C: np.ndarray):
    """labels_i = argmin_c sum_r (F_ir - C_cr)^2 (float64, columns summed in
    order, each square rounded before the add), lowest c on ties.
    Returns (labels int32, min squared distance float64)."""
    F = np.asarray(F, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    n, r = F.shape
    k = C.shape[0]
    D = np.zeros((n, k))
    for c in range(k):
        d = np.zeros(n)
        for col in range(r):
            diff = F[:, col] - C[c, col]
            sq = diff * diff
            d = d + sq
        D[:, c] = d
    labels = np.argmin(D, axis=1).astype(np.int32)   # first minimum = lowest index
    return labels, D[np.arange(n), labels]


def kmeans_update(F: np.ndarray, labels: np.ndarray, C_prev: np.ndarray):
    """(C_new, counts): mean of the members of each cluster in float64; an
    empty cluster keeps C_prev."""
    F = np.asarray(F, dtype=np.float64)
    k, r = C_prev.shape
    counts = np.bincount(labels, minlength=k).astype(np.int64)
    sums = np.zeros((k, r))
    np.add.at(sums, labels, F)
    C = np.array(C_prev, dtype=np.float64, copy=True)
    ne = counts > 0
    C[ne] = sums[ne] / counts[ne, None]
    return C, counts


def kmeans_lloyd(F, C0, iters: int, centroid_dtype=np.float32):
    """``iters`` Lloyd iterations (assign, then update), then a final
    assignment against the last centroids; returns (labels, C).  Centroids are
    stored in ``centroid_dtype`` between iterations (float32 in the library's
    interface; pass np.float64 for a pure float64 run)."""
    C = np.asarray(C0, dtype=centroid_dtype)
    for _ in range(iters):
        labels, _ = kmeans_assign(F, C)
        C, _ = kmeans_update(F, labels, C)
        C = C.astype(centroid_dtype)
    labels, _ = kmeans_assign(F, C)
    return labels, C
