"""GPU parity of the moments, eigenvalue count and dichotomy (Sec. 3.2), row
normalisation and k-means (Sec. 2.2 step 4, Sec. 4.1 step 6) against the
FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_1509_08863_amd as asc

from gpu_util import DEV, upload_graph, block_f32, block_bf16, scalar, host, rel_fro, to_dev

pytestmark = pytest.mark.gpu


def _setup(g, p):
    w = g.weights_or_ones().astype(np.float64)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, w)
    lmax = 1.01 * oracle.lambda_max_exact(L)
    return L, lmax


@pytest.mark.parametrize("p", [0, 1, 2, 5, 50, 51])
@pytest.mark.parametrize("r", [4, 32, 33])
def test_moments_match_oracle(p, r):
    g = W.workload_graph(1)
    L, lmax = _setup(g, p)
    G = upload_graph(g)
    Rs, R64 = W.signals(g.n, r, 11)
    mu = host(asc.cheb_moments(G, scalar(lmax), p, block_f32(Rs)))
    ref = oracle.moments(L, lmax, p, R64)
    # mu_0 = |R|^2 ~ n; float32 states give absolute errors ~1e-6 of mu_0
    assert np.max(np.abs(mu - ref)) <= 1e-5 * ref[0]
    # the count is a weighted sum of moments; compare it at a few cut-offs
    for frac in (0.05, 0.17, 0.5):
        c_gpu = float(np.dot(oracle.cheb_coeffs(frac * lmax, lmax, p), mu))
        c_ref = oracle.eigcount_from_moments(ref, frac * lmax, lmax)
        assert abs(c_gpu - c_ref) <= 1e-5 * ref[0] / np.sqrt(max(p, 1))


def test_dichotomy_on_oracle_moments_is_exact():
    # identical float64 moments in -> identical bisection decisions
    g = W.workload_graph(1)
    L, lmax = _setup(g, 50)
    R64 = W.signals(g.n, 32, 4)[1]
    mu = oracle.moments(L, lmax, 50, R64)
    est_ref, traj_ref = oracle.dichotomy(lambda lc: oracle.eigcount_from_moments(mu, lc, lmax), lmax, 10, 12)
    lam, traj = asc.eigcount_dichotomy(to_dev(mu), scalar(lmax), 10, 12)
    traj = host(traj)
    np.testing.assert_array_equal(traj[:, 0], traj_ref[:, 0])
    np.testing.assert_allclose(traj[:, 1], traj_ref[:, 1], rtol=1e-12, atol=1e-12)
    assert host(lam)[0] == est_ref


def _traj_agree(traj, traj_ref, k, tol):
    """Trajectories agree until the first near tie |count - (k - 1/2)| <= tol."""
    for s in range(len(traj_ref)):
        if abs(traj_ref[s, 1] - (k - 0.5)) <= tol:
            return True
        assert traj[s, 0] == traj_ref[s, 0], s
        assert abs(traj[s, 1] - traj_ref[s, 1]) <= tol, s
    return True


@pytest.mark.parametrize("literal", [False, True])
def test_lambda_k_matches_oracle(literal):
    g = W.workload_graph(1)
    L, lmax = _setup(g, 50)
    G = upload_graph(g)
    Rs, R64 = W.signals(g.n, 32, 6)
    est_ref, traj_ref = oracle.dichotomy_moments(L, lmax, 10, 50, 12, R64)
    lam, traj = asc.eigcount_lambda_k(G, scalar(lmax), 10, 50, 12, block_f32(Rs), literal=literal)
    _traj_agree(host(traj), traj_ref, 10, 1e-3)


def test_large_gap_lambda_k():
    k, m = 6, 16
    g = W.cliques(k, m, bridges=True)
    L, lmax = _setup(g, 120)
    lam_all = np.linalg.eigvalsh(L.toarray())
    G = upload_graph(g)
    Rs, _ = W.signals(g.n, 64, 2)
    lam, _ = asc.eigcount_lambda_k(G, scalar(lmax), k, 120, 14, block_f32(Rs))
    assert lam_all[k - 1] < host(lam)[0] < lam_all[k]


def test_normalize_matches_oracle():
    rng = np.random.default_rng(5)
    Y = rng.standard_normal((3000, 50)).astype(np.float32)
    Y[7] = 0
    Yd = block_f32(Y, 52)
    norms = asc.normalize_features(Yd)
    F, nrm = oracle.normalize_rows(Y.astype(np.float64))
    np.testing.assert_allclose(host(Yd), F, rtol=2e-7, atol=1e-30)
    np.testing.assert_allclose(host(norms), nrm, rtol=1e-7)
    assert np.all(host(Yd)[7] == 0)


@pytest.mark.parametrize("n,r,k", [(5000, 64, 20), (1000, 96, 50), (333, 7, 3), (64, 130, 200), (1000, 130, 7),
                                   (777, 5, 2), (2000, 40, 32), (2000, 40, 33), (1500, 256, 32), (301, 3, 1),
                                   (1001, 32, 100), (3, 40, 40), (70, 64, 64), (513, 100, 80)])
def test_kmeans_assign_bit_exact(n, r, k):
    rng = np.random.default_rng(n + k)
    F = rng.standard_normal((n, r)).astype(np.float32)
    C = rng.standard_normal((k, r)).astype(np.float32)
    if k > 1:
        C[1] = C[0]  # an exact tie: lowest index wins
    labels, dist2 = asc.kmeans_assign(block_f32(F), to_dev(C))
    lab_ref, d_ref = oracle.kmeans_assign(F, C)
    np.testing.assert_array_equal(host(labels), lab_ref)
    np.testing.assert_array_equal(host(dist2), d_ref.astype(np.float32))
    # without the distance output (the float64 distance is skipped where the
    # candidate is certain): the same labels
    labels_nd, none = asc.kmeans_assign(block_f32(F), to_dev(C), dist=False)
    assert none is None
    np.testing.assert_array_equal(host(labels_nd), lab_ref)


@pytest.mark.parametrize("n,r,k", [(5000, 64, 20), (20000, 96, 50), (100, 8, 7), (3000, 300, 10), (2000, 40, 3)])
def test_kmeans_update_matches_oracle(n, r, k):
    rng = np.random.default_rng(k)
    F = rng.standard_normal((n, r)).astype(np.float32)
    lab = rng.integers(0, k, n).astype(np.int32)
    lab[lab == 2] = 0  # an empty cluster keeps its centroid
    C0 = rng.standard_normal((k, r)).astype(np.float32)
    Cd = to_dev(C0.copy())
    counts = asc.kmeans_update(block_f32(F), to_dev(lab), Cd)
    C_ref, cnt_ref = oracle.kmeans_update(F.astype(np.float64), lab, C0.astype(np.float64))
    np.testing.assert_array_equal(host(counts), cnt_ref)
    got = host(Cd)
    ref32 = C_ref.astype(np.float32)
    ulp = np.spacing(np.abs(ref32))
    assert np.all(np.abs(got - ref32) <= ulp)
    np.testing.assert_array_equal(got[2], C0[2])


def test_kmeans_init_rows():
    F = np.random.default_rng(1).standard_normal((100, 12)).astype(np.float32)
    rows = np.array([3, 50, 99], dtype=np.int32)
    C = asc.kmeans_init_rows(block_f32(F), to_dev(rows))
    np.testing.assert_array_equal(host(C), F[rows])


@pytest.mark.parametrize("r,p", [(32, 50), (33, 51), (8, 1)])
def test_one_pass_lambda_k_filter(r, p):
    g = W.workload_graph(1)
    L, lmax = _setup(g, p)
    G = upload_graph(g)
    Rs, R64 = W.signals(g.n, r, 13)
    k, steps = 10, 12
    Y, lam, traj, co, states = asc.lambda_k_filter(G, scalar(lmax), k, p, steps, block_f32(Rs))
    # the same moments and decisions as the two-pass entry points
    lam2, traj2 = asc.eigcount_lambda_k(G, scalar(lmax), k, p, steps, block_f32(Rs))
    np.testing.assert_array_equal(host(traj), host(traj2))
    Y2 = asc.cheb_filter(G, scalar(lmax), asc.cheb_coeffs(lam2, scalar(lmax), p), block_f32(Rs))
    assert rel_fro(host(Y), host(Y2)) <= 1e-6
    np.testing.assert_array_equal(host(co), host(asc.cheb_coeffs(lam, scalar(lmax), p))[0])
    # against the oracle (same decisions up to a near tie)
    est_ref, traj_ref = oracle.dichotomy_moments(L, lmax, k, p, steps, R64)
    _traj_agree(host(traj), traj_ref, k, 1e-3)
    if np.all(np.abs(traj_ref[:, 1] - (k - 0.5)) > 1e-3):
        Yref = oracle.cheb_filter(L, lmax, oracle.cheb_coeffs(est_ref, lmax, p), R64)
        assert rel_fro(host(Y), Yref) <= 1e-5


@pytest.mark.parametrize("n,r,k", [(4000, 96, 50), (3000, 24, 10), (2500, 128, 64), (1000, 4, 2)])
def test_kmeans_assign_near_ties_stay_exact(n, r, k):
    # rows at midpoints of centroid pairs (plus noise far below the float32
    # error of the dot-product form), exact midpoints, duplicated centroids
    # and a non-finite row: the matrix-core proposals cannot certify these,
    # the float64 rerun decides, and the labels equal the definition's
    rng = np.random.default_rng(r + k)
    C = rng.standard_normal((k, r)).astype(np.float32)
    C[k - 1] = C[0]
    a = rng.integers(0, k, n)
    b = rng.integers(0, k, n)
    F = (0.5 * (C[a].astype(np.float64) + C[b].astype(np.float64))).astype(np.float32)
    F[: n // 2] += (rng.standard_normal((n // 2, r)) * 1e-6).astype(np.float32)
    F[n // 3] = np.nan
    labels, dist2 = asc.kmeans_assign(block_f32(F), to_dev(C))
    ok = np.all(np.isfinite(F), axis=1)
    lab_ref, d_ref = oracle.kmeans_assign(F[ok], C)
    np.testing.assert_array_equal(host(labels)[ok], lab_ref)
    np.testing.assert_array_equal(host(dist2)[ok], d_ref.astype(np.float32))
    labels_nd, _ = asc.kmeans_assign(block_f32(F), to_dev(C), dist=False)
    np.testing.assert_array_equal(host(labels_nd), host(labels))
