"""K-nearest-neighbour similarity graph (Sec. 5: a K-nearest-neighbours graph
with K ~ log N), union-symmetrised, with the squared edge lengths that the
Gaussian kernel w = exp(-d^2 / sigma^2) of Sec. 2.2 turns into weights.
Test infrastructure only.

Readings taken here:
  * the neighbours of point i are the K points j != i of least squared
    Euclidean distance |x_i - x_j|^2, computed in float64 from the given
    float32 coordinates, summed over the coordinates in order with every
    square rounded before the add; equal distances go to the lower index;
  * the graph keeps the edge {i, j} when j is a neighbour of i or i one of j
    (union), stored in both directions with its float64 distance rounded to
    float32.

Pinned by (tests/test_oracle_knn.py): a pure-Python brute force on small
point sets with duplicated points (ties); scipy's cKDTree on generic data
(the same sets, distances to 1e-12); the union graph against a set-based
construction, its symmetry and sortedness, and the complete graph when
K >= N - 1.
"""
from __future__ import annotations

import numpy as np


def sqdist_to(X, i, idx=None) -> np.ndarray:
    """|x_i - x_j|^2 for j in idx (all rows by default), float64, the
    coordinates added in order."""
    X = np.asarray(X, dtype=np.float64)
    Y = X if idx is None else X[np.asarray(idx)]
    acc = np.zeros(Y.shape[0])
    for c in range(X.shape[1]):
        t = Y[:, c] - X[i, c]
        acc = acc + t * t
    return acc


def knn_bruteforce(X, K):
    """(idx [n][K], d2 [n][K]) in order of (distance, index)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    idx = np.zeros((n, K), dtype=np.int64)
    d2 = np.zeros((n, K))
    j = np.arange(n)
    for i in range(n):
        d = sqdist_to(X, i)
        d[i] = np.inf
        o = np.lexsort((j, d))[:K]
        idx[i], d2[i] = o, d[o]
    return idx, d2


def knn(X, K, extra: int = 16):
    """Same result as knn_bruteforce for large n: a k-d tree proposes K + extra
    candidates per point, their float64 distances are recomputed as above and
    sorted; a row whose K-th distance is not below the tree's last candidate
    distance (minus a 1e-9 relative margin) is redone by brute force."""
    from scipy.spatial import cKDTree
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    m = min(n, K + extra + 1)
    dist, nb = cKDTree(X).query(X, k=m, workers=-1)
    idx = np.zeros((n, K), dtype=np.int64)
    d2 = np.zeros((n, K))
    jall = np.arange(n)
    for i in range(n):
        cand = nb[i][nb[i] != i]
        d = sqdist_to(X, i, cand)
        o = np.lexsort((cand, d))
        if len(cand) >= K and (m >= n or d[o[K - 1]] < dist[i, -1] ** 2 * (1.0 - 1e-9)):
            idx[i], d2[i] = cand[o[:K]], d[o[:K]]
        else:
            dd = sqdist_to(X, i)
            dd[i] = np.inf
            oo = np.lexsort((jall, dd))[:K]
            idx[i], d2[i] = oo, dd[oo]
    return idx, d2


def union_graph(n, idx, X):
    """CSR (row_ptr int32, col_idx int32, d2 float32) of the union of the
    directed neighbour lists, columns increasing in every row."""
    X = np.asarray(X, dtype=np.float64)
    idx = np.asarray(idx, dtype=np.int64)
    K = idx.shape[1]
    src = np.repeat(np.arange(n), K)
    dst = idx.reshape(-1)
    u = np.concatenate([src, dst])
    v = np.concatenate([dst, src])
    key = np.unique(u * n + v)
    rows, cols = key // n, key % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    d2 = np.zeros(len(cols))
    for c in range(X.shape[1]):
        t = X[cols, c] - X[rows, c]
        d2 = d2 + t * t
    return row_ptr.astype(np.int32), cols.astype(np.int32), d2.astype(np.float32)
