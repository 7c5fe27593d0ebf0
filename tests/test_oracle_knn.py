"""Pins of the kNN-graph oracle (Sec. 5 graph construction)."""
import numpy as np
import pytest

from oracle import knn
import oracle
import workloads as W


def _py_knn(X, K):
    n = len(X)
    out = []
    for i in range(n):
        cand = []
        for j in range(n):
            if j == i:
                continue
            s = 0.0
            for c in range(len(X[i])):
                t = float(X[j][c]) - float(X[i][c])
                s = s + t * t
            cand.append((s, j))
        cand.sort()
        out.append(cand[:K])
    return out


@pytest.mark.parametrize("seed", range(4))
def test_bruteforce_against_pure_python_with_ties(seed):
    rng = np.random.default_rng(seed)
    X = rng.integers(0, 4, size=(30, 3)).astype(np.float32)  # many equal distances
    X[5] = X[7]  # a duplicated point: distance 0 both ways
    K = 6
    idx, d2 = knn.knn_bruteforce(X, K)
    ref = _py_knn(X.tolist(), K)
    for i in range(len(X)):
        assert [j for _, j in ref[i]] == idx[i].tolist()
        assert [s for s, _ in ref[i]] == d2[i].tolist()


def test_tree_path_equals_bruteforce():
    x, _ = W.gmm2d_points(3000, 6, 5)
    X = np.concatenate([x, np.random.default_rng(1).standard_normal((3000, 3))], axis=1).astype(np.float32)
    K = 9
    a_idx, a_d2 = knn.knn(X, K)
    full_idx, full_d2 = knn.knn_bruteforce(X, K)
    np.testing.assert_array_equal(a_idx, full_idx)
    np.testing.assert_array_equal(a_d2, full_d2)


def test_against_scipy_kdtree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(2)
    X = rng.standard_normal((2000, 16)).astype(np.float32)
    K = 10
    idx, d2 = knn.knn(X, K)
    dist, nb = cKDTree(X.astype(np.float64)).query(X.astype(np.float64), k=K + 1)
    np.testing.assert_allclose(d2, dist[:, 1:] ** 2, rtol=1e-12)
    for i in range(0, 2000, 7):
        assert set(idx[i]) == set(nb[i, 1:])


def test_union_graph():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((500, 4)).astype(np.float32)
    K = 5
    idx, _ = knn.knn_bruteforce(X, K)
    rp, ci, d2 = knn.union_graph(500, idx, X)
    oracle.check_graph(500, rp, ci, None)  # sorted, symmetric, no self-loops
    edges = set()
    for i in range(500):
        for j in idx[i]:
            edges.add((i, int(j)))
            edges.add((int(j), i))
    got = {(i, int(j)) for i in range(500) for j in ci[rp[i]:rp[i + 1]]}
    assert got == edges
    assert np.all(np.diff(rp) >= K)
    rows = np.repeat(np.arange(500), np.diff(rp))
    for e in range(0, len(ci), 37):
        assert d2[e] == np.float32(knn.sqdist_to(X, rows[e], [ci[e]])[0])
    # K >= n - 1: the complete graph
    Xs = X[:12]
    idx2, _ = knn.knn_bruteforce(Xs, 11)
    rp2, ci2, _ = knn.union_graph(12, idx2, Xs)
    assert np.all(np.diff(rp2) == 11)
