"""Pins of the oracle's row normalisation and k-means (Sec. 2.2 step 4, Sec. 4.1 step 6)."""
import itertools

import numpy as np
import pytest

import oracle
import workloads as W


def test_normalize_rows():
    Y = np.random.default_rng(1).standard_normal((50, 7))
    Y[3] = 0
    F, nrm = oracle.normalize_rows(Y)
    np.testing.assert_allclose(np.linalg.norm(F[np.arange(50) != 3], axis=1), 1, atol=1e-15)
    assert np.all(F[3] == 0) and nrm[3] == 0
    np.testing.assert_allclose(F * nrm[:, None], Y, atol=1e-15)


def _brute_assign(F, C):
    labels = []
    for i in range(F.shape[0]):
        best, bc = None, -1
        for c in range(C.shape[0]):
            d = sum((float(F[i, r]) - float(C[c, r])) ** 2 for r in range(F.shape[1]))
            if best is None or d < best:
                best, bc = d, c
        labels.append(bc)
    return np.array(labels)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_assign_brute_force(seed):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((40, 5)).astype(np.float32)
    C = rng.standard_normal((6, 5)).astype(np.float32)
    lab, d = oracle.kmeans_assign(F, C)
    np.testing.assert_array_equal(lab, _brute_assign(F, C))
    ref = np.min(((F[:, None, :].astype(float) - C[None].astype(float)) ** 2).sum(-1), axis=1)
    np.testing.assert_allclose(d, ref, rtol=1e-14)


def test_assign_ties_lowest_index():
    F = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, 0.0]])
    C = np.array([[1.0, 0.0], [-1.0, 0.0], [0.0, 1.0], [0.0, 0.0], [0.0, 0.0]])
    lab, _ = oracle.kmeans_assign(F, C)
    # row 0: centroids 3 and 4 tie at 0 -> 3; row 2: centroids 0 and 3 tie at 0.25 -> 0
    np.testing.assert_array_equal(lab, [3, 0, 0])


def test_update_mean_and_empty():
    rng = np.random.default_rng(4)
    F = rng.standard_normal((30, 3))
    lab = rng.integers(0, 4, 30)
    lab[lab == 2] = 0  # cluster 2 empty
    Cp = rng.standard_normal((4, 3))
    C, cnt = oracle.kmeans_update(F, lab, Cp)
    for c in range(4):
        rows = [F[i] for i in range(30) if lab[i] == c]
        assert cnt[c] == len(rows)
        if rows:
            np.testing.assert_allclose(C[c], np.mean(rows, axis=0), rtol=1e-14)
        else:
            np.testing.assert_array_equal(C[c], Cp[c])


def test_disjoint_cliques_recovered():
    # exact ideal-filter features of disjoint cliques are constant per block,
    # so k-means from one seed row per block recovers the blocks exactly
    k, m = 5, 8
    g = W.cliques(k, m)
    L = oracle.laplacian_dense(g.n, g.row_ptr, g.col_idx, g.w)
    lam, chi = oracle.dense_spectrum(L)
    R = W.signals(g.n, 2 * k, 3)[1]
    Fe = oracle.ideal_filter(lam, chi, 0.5, R)
    F, _ = oracle.normalize_rows(Fe)
    init = np.arange(k) * m + 3
    lab, _ = oracle.kmeans_lloyd(F, F[init], 5, np.float64)
    for a, b in itertools.combinations(range(g.n), 2):
        assert (lab[a] == lab[b]) == (g.labels[a] == g.labels[b])
