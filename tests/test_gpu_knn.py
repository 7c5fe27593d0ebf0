"""GPU parity of the K-nearest-neighbour graph construction (Sec. 5) against
the exact float64 oracle: neighbour lists, distances and the union graph are
compared element by element."""
import numpy as np
import pytest

import oracle
from oracle import knn as oknn
import workloads as W
import paper_1509_08863_amd as asc

from gpu_util import host, to_dev

pytestmark = pytest.mark.gpu


def _check(X, K, ref=None, ld=None):
    Xd = to_dev(X.astype(np.float32))
    if ld is not None:  # rows ld floats apart (columns past d hold other values)
        buf = to_dev(np.full((len(X), ld), 7.5, np.float32))
        buf[:, :X.shape[1]] = Xd
        Xd = buf[:, :X.shape[1]]
    out = asc.knn_graph(Xd, K)
    idx, d2 = ref if ref is not None else oknn.knn_bruteforce(X, K)
    np.testing.assert_array_equal(host(out["nbr"]), idx)
    np.testing.assert_array_equal(host(out["nbr_d2"]), d2)
    rp, ci, dd = oknn.union_graph(len(X), idx, X)
    np.testing.assert_array_equal(host(out["row_ptr"]), rp)
    np.testing.assert_array_equal(host(out["col_idx"]), ci)
    np.testing.assert_array_equal(host(out["d2"]), dd)
    return out


@pytest.mark.parametrize("n,d,K", [(300, 3, 6), (1000, 16, 10), (777, 5, 1), (513, 17, 32), (129, 64, 7),
                                   (2000, 2, 9), (40, 1, 3), (33, 33, 32), (1000, 20, 10), (700, 8, 5)])
def test_knn_matches_oracle(n, d, K):
    rng = np.random.default_rng(n + d + K)
    if d <= 3:
        X = rng.integers(0, 5, size=(n, d)).astype(np.float32)  # many exact ties
    else:
        X = rng.standard_normal((n, d)).astype(np.float32) * 3.0
    X[7] = X[3]  # a duplicated point
    _check(X, K)


def test_knn_smallest_and_complete():
    X = np.random.default_rng(1).standard_normal((9, 4)).astype(np.float32)
    out = _check(X, 8)  # K = n - 1: every other point
    assert np.all(np.diff(host(out["row_ptr"])) == 8)
    _check(X[:2], 1)


def test_knn_far_offset_points_use_the_fallback_and_stay_exact():
    # large norms make the float32 proposals too coarse to certify: the rows
    # go through the float64 scan and the result is still exact
    rng = np.random.default_rng(2)
    X = (rng.standard_normal((1500, 8)) * 0.05 + 200.0).astype(np.float32)
    out = _check(X, 10)
    assert host(out["fallback_rows"])[0] > 0


def test_knn_nonfinite_point_is_isolated():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((400, 6)).astype(np.float32)
    X[11, 2] = np.nan
    out = asc.knn_graph(to_dev(X), 5)
    nbr = host(out["nbr"])
    assert np.all(nbr[11] == -1)
    assert not np.any(nbr == 11)
    keep = np.arange(400) != 11
    idx, d2 = oknn.knn_bruteforce(X[keep], 5)
    # renumber the oracle's indices to the full set
    full = np.arange(400)[keep]
    np.testing.assert_array_equal(nbr[keep], full[idx])
    rp = host(out["row_ptr"])
    assert rp[12] == rp[11]  # no edges at the non-finite point


def test_knn_full_size_gaussian_mixture_and_weights():
    # the gradient workload's point set: 2e5 points of a 16-D, 20-component
    # mixture, K = 10; the oracle proposes with a k-d tree and decides in float64
    x, _ = W.gmm_points(200_000, 16, 20, W.workload_seeds(5)["graph"])
    X = x.astype(np.float32)
    ref = oknn.knn(X, 10)
    out = _check(X, 10, ref)
    print("fallback rows", host(out["fallback_rows"])[0])
    w = asc.gauss_weights(out["d2"], 2.0)
    rp, ci, dd = oknn.union_graph(len(X), ref[0], X)
    np.testing.assert_allclose(host(w), oracle.gauss_weights(dd.astype(np.float64), 2.0), rtol=1e-7)


@pytest.mark.parametrize("d,ld", [(18, 20), (18, 24), (13, 16), (16, 20)])
def test_knn_rows_with_a_wider_leading_dimension(d, ld):
    # 16-byte rows with padding past d (the padding holds other values, which
    # must not reach the distances), and quads past d never read
    X = np.random.default_rng(d * ld).standard_normal((900, d)).astype(np.float32) * 2.0
    _check(X, 9, ld=ld)
