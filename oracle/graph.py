"""Combinatorial Laplacian L = S - W (Sec. 2.1).  Test infrastructure only.

W is given as CSR (row_ptr, col_idx, w) with both directions stored; S is
diagonal with s_i = sum_{j != i} W_ij, the strength of node i.

Also the normalised Laplacian L_n = I - S^{-1/2} W S^{-1/2} of the footnote
of Sec. 2.1.

Pinned by: L 1 = 0, L symmetric, smallest eigenvalue >= 0 and dim ker L equal to
the number of connected components (tests/test_oracle_graph.py); L_n by the
closed-form spectra of complete graphs and cycles, the eigenvalue 2 of
bipartite graphs, spectrum inside [0, 2], and L_n S^{1/2} 1 = 0
(tests/test_oracle_graph_spectrum.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _w64(nnz, w):
    return np.ones(nnz) if w is None else np.asarray(w, dtype=np.float64)


def adjacency_sparse(n, row_ptr, col_idx, w=None) -> sp.csr_matrix:
    """W as a float64 scipy CSR matrix (entries exactly as stored)."""
    return sp.csr_matrix((_w64(len(col_idx), w), np.asarray(col_idx), np.asarray(row_ptr)), shape=(n, n))


def strength(n, row_ptr, col_idx, w=None) -> np.ndarray:
    """s_i = sum_j W_ij over the stored entries of row i (float64)."""
    W = adjacency_sparse(n, row_ptr, col_idx, w)
    return np.asarray(W.sum(axis=1)).reshape(-1)


def laplacian_sparse(n, row_ptr, col_idx, w=None) -> sp.csr_matrix:
    """L = S - W (float64 sparse)."""
    W = adjacency_sparse(n, row_ptr, col_idx, w)
    s = np.asarray(W.sum(axis=1)).reshape(-1)
    return (sp.diags(s) - W).tocsr()


def laplacian_normalized(n, row_ptr, col_idx, w=None) -> sp.csr_matrix:
    """L_n = I - S^{-1/2} W S^{-1/2} (footnote of Sec. 2.1), float64 sparse;
    a node of zero strength has S^{-1/2} = 0 there (its row of L_n is e_i)."""
    W = adjacency_sparse(n, row_ptr, col_idx, w)
    s = np.asarray(W.sum(axis=1)).reshape(-1)
    dinv = np.zeros(n)
    dinv[s > 0] = 1.0 / np.sqrt(s[s > 0])
    D = sp.diags(dinv)
    return (sp.identity(n, format="csr") - D @ W @ D).tocsr()


def laplacian_dense(n, row_ptr, col_idx, w=None) -> np.ndarray:
    return laplacian_sparse(n, row_ptr, col_idx, w).toarray()


def check_graph(n, row_ptr, col_idx, w=None) -> None:
    """Raise ValueError unless W is a valid undirected weighted graph as the
    paper defines it: W_ij = W_ji >= 0, no self-loops; CSR sorted in-range."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    if row_ptr[0] != 0 or row_ptr[-1] != len(col_idx) or np.any(np.diff(row_ptr) < 0):
        raise ValueError("bad row_ptr")
    if len(col_idx) and (col_idx.min() < 0 or col_idx.max() >= n):
        raise ValueError("column index out of range")
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    if np.any(rows == col_idx):
        raise ValueError("self-loop")
    same_row = rows[1:] == rows[:-1]
    if np.any(col_idx[1:][same_row] <= col_idx[:-1][same_row]):
        raise ValueError("columns not strictly increasing")
    ww = _w64(len(col_idx), w)
    if np.any(~np.isfinite(ww)) or np.any(ww < 0):
        raise ValueError("weights must be finite and >= 0")
    W = adjacency_sparse(n, row_ptr, col_idx, w)
    if abs(W - W.T).max() != 0 if W.nnz else False:
        raise ValueError("W not symmetric")
