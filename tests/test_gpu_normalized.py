"""GPU parity of the normalised-Laplacian variant (footnote of Sec. 2.1):
L_n = I - S^-1/2 W S^-1/2 through the same filter, eigenvalue count and
clustering entry points, against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_1509_08863_amd as asc

from gpu_util import upload_graph, block_f32, scalar, host, rel_fro, to_dev

pytestmark = pytest.mark.gpu


def _ln(g):
    return oracle.laplacian_normalized(g.n, g.row_ptr, g.col_idx, None if g.w is None else g.w.astype(np.float64))


@pytest.mark.parametrize("make", [lambda: W.random_weighted(700, 0.02, 3, isolated=5),
                                  lambda: W.workload_graph(1), lambda: W.cliques(6, 15, bridges=True)])
def test_normalized_weights_and_filter(make):
    g = make()
    G = upload_graph(g)
    Gn = asc.graph_normalized(G)
    Ln = _ln(g)
    # off-diagonal entries of L_n are -w'_e
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    ref = -np.asarray(Ln[rows, g.col_idx]).reshape(-1)
    np.testing.assert_allclose(host(Gn.w), ref, rtol=2e-7, atol=0)
    np.testing.assert_array_equal(host(Gn.strength), np.ones(g.n))
    r, p = 20, 60
    Rs, R64 = W.signals(g.n, r, 8)
    lam = np.linalg.eigvalsh(Ln.toarray())
    assert lam.max() <= 2.0 + 1e-12
    a = oracle.cheb_coeffs(0.3, 2.0, p)
    Y = host(asc.cheb_filter(Gn, scalar(2.0), to_dev(a), block_f32(Rs)))
    # the oracle applies its own L_n to the same float32-rounded signals
    Yref = oracle.cheb_filter(Ln, 2.0, a, R64)
    assert rel_fro(Y, Yref) <= 1e-5


def test_normalized_lmax_estimate_and_lambda_k():
    g = W.workload_graph(1)
    Gn = asc.graph_normalized(upload_graph(g))
    Ln = _ln(g)
    lam = np.linalg.eigvalsh(Ln.toarray())
    lm = asc.lmax_estimate(Gn, to_dev(W.start_vector(g.n, 3)), 80, host=True)[1]
    assert lam[-1] <= lm <= 2.0
    k, p, steps = 10, 80, 12
    Rs, R64 = W.signals(g.n, 32, 9)
    est_ref, traj_ref = oracle.dichotomy_moments(Ln, 2.0, k, p, steps, R64)
    Y, lamk, traj, co, _ = asc.lambda_k_filter(Gn, scalar(2.0), k, p, steps, block_f32(Rs))
    traj = host(traj)
    for s in range(steps):
        if abs(traj_ref[s, 1] - (k - 0.5)) <= 1e-3:
            break
        assert traj[s, 0] == traj_ref[s, 0]
        assert abs(traj[s, 1] - traj_ref[s, 1]) <= 1e-3


def test_normalized_pipeline_recovers_cliques():
    # Ng-Jordan-Weiss style: normalised Laplacian, filtered signals, row
    # normalisation, k-means
    k, m = 5, 30
    g = W.cliques(k, m, bridges=True)
    Gn = asc.graph_normalized(upload_graph(g))
    Rs, _ = W.signals(g.n, 16, 4)
    Y, lamk, _, _, _ = asc.lambda_k_filter(Gn, scalar(2.0), k, 100, 14, block_f32(Rs))
    asc.normalize_features(Y)
    rows = np.array([0, m, 2 * m, 3 * m, 4 * m], dtype=np.int32) + 3
    C = asc.kmeans_init_rows(Y, to_dev(rows))
    for _ in range(10):
        lab, _ = asc.kmeans_assign(Y, C)
        asc.kmeans_update(Y, lab, C)
    lab, _ = asc.kmeans_assign(Y, C)
    assert oracle.ari(host(lab), g.labels) == 1.0
