"""GPU parity of the stability measure gamma(k) (Sec. 4.3, Eq. stab) and of
the adjusted Rand index against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_1509_08863_amd as asc

from gpu_util import upload_graph, block_f32, block_bf16, scalar, host, to_dev

pytestmark = pytest.mark.gpu


def _pools(Rs, J, eta_max):
    R64 = Rs.astype(np.float64)
    return [R64[:, j * eta_max:(j + 1) * eta_max] for j in range(J)]


def test_ari_pairs_match_oracle():
    rng = np.random.default_rng(4)
    n, k = 3000, 7
    base = rng.integers(0, k, n)
    labs = [base, rng.permutation(k)[base], np.where(rng.random(n) < 0.8, base, rng.integers(0, k, n)),
            rng.integers(0, k, n), np.zeros(n, np.int64)]
    L = np.stack(labs).astype(np.int32)
    ari, mean = asc.ari_pairs(to_dev(L), k)
    ref = oracle.ari_pairs(labs)
    np.testing.assert_allclose(host(ari), ref, rtol=1e-13, atol=1e-15)
    assert host(ari)[0] == 1.0  # a relabelling
    assert host(mean)[0] == pytest.approx(float(np.mean(ref)), rel=1e-13)
    # strided rows (ldl > n) and the degenerate one-cluster pair
    Lp = np.zeros((2, n + 5), np.int32)
    ari2, _ = asc.ari_pairs(to_dev(Lp)[:, :n], 1)
    assert host(ari2)[0] == 1.0


@pytest.mark.parametrize("k", [1, 2, 5, 127, 128])
def test_ari_cluster_count_limits(k):
    rng = np.random.default_rng(k)
    n = 6000
    base = rng.integers(0, k, n)
    labs = [base, np.where(rng.random(n) < 0.6, base, rng.integers(0, k, n)), rng.integers(0, k, n)]
    ari, _ = asc.ari_pairs(to_dev(np.stack(labs).astype(np.int32)), k)
    np.testing.assert_allclose(host(ari), oracle.ari_pairs(labs), rtol=1e-13, atol=1e-15)


def test_ari_skips_invalid_labels_and_flags_them():
    rng = np.random.default_rng(5)
    n, k = 1000, 4
    a = rng.integers(0, k, n).astype(np.int32)
    b = rng.integers(0, k, n).astype(np.int32)
    b[17] = k  # out of range
    ari, _ = asc.ari_pairs(to_dev(np.stack([a, b])), k)
    flags = asc.read_flags(asc.ari_pairs.last_ws, raise_on_error=False)
    assert flags & 8
    keep = np.ones(n, bool)
    keep[17] = False
    assert host(ari)[0] == pytest.approx(oracle.ari(a[keep], b[keep]), rel=1e-13, abs=1e-15)


def _run(g, ks, etas, J, reps, p, steps, iters, seed_sig, seed_rows, lmax=None):
    eta_max = max(etas)
    Rs, _ = W.stability_pools(g.n, J, eta_max, seed_sig)
    rows = W.stability_init_rows(g.n, ks, J, reps, seed_rows)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, g.weights_or_ones().astype(np.float64))
    if lmax is None:
        lmax = 1.01 * oracle.lambda_max_exact(L)
    G = upload_graph(g)
    out = asc.stability(G, scalar(lmax), ks[0], ks[-1], etas, J, reps, p, steps, iters, block_f32(Rs), eta_max,
                        to_dev(rows))
    res = {k_: host(v) for k_, v in out.items()}
    return res, L, lmax, _pools(Rs, J, eta_max), rows


def _traj_agree(traj, traj_ref, k, tol=1e-3):
    for s in range(len(traj_ref)):
        if abs(traj_ref[s, 1] - (k - 0.5)) <= tol:
            return False
        assert traj[s, 0] == traj_ref[s, 0], s
        assert abs(traj[s, 1] - traj_ref[s, 1]) <= tol, s
    return True


def test_stability_cliques_matches_oracle_exactly():
    g = W.cliques(5, 20, bridges=True)
    ks = [3, 4, 5, 6, 7]
    etas = [2 * k for k in ks]
    J, reps, p, steps, iters = 5, 5, 60, 12, 10
    res, L, lmax, pools, rows = _run(g, ks, etas, J, reps, p, steps, iters, 11, 12)
    ref = oracle.stability(L, lmax, ks, etas, pools, p, steps, rows, iters)
    for q, k in enumerate(ks):
        for j in range(J):
            _traj_agree(res["traj"][q, j], ref["traj"][q][j], k)
            np.testing.assert_array_equal(res["labels"][q, j], ref["labels"][q][j])
        np.testing.assert_allclose(res["ari"][q], ref["ari"][q], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(res["gamma"], ref["gamma"], rtol=1e-13, atol=1e-15)
    assert res["gamma"][2] == 1.0 and int(np.argmax(res["gamma"])) == 2


def test_stability_planar_mixture_matches_oracle():
    # a reduced version of the benchmark workload: 2000 points of a planar
    # 6-Gaussian mixture, kNN with K = round(ln N), k = 4..8
    x, z = W.gmm2d_points(2000, 6, 77)
    g = W.knn_graph(x, int(round(np.log(2000))))
    ks = [4, 5, 6, 7, 8]
    etas = [2 * k for k in ks]
    J, reps, p, steps, iters = 4, 3, 80, 12, 15
    res, L, lmax, pools, rows = _run(g, ks, etas, J, reps, p, steps, iters, 21, 22)
    ref = oracle.stability(L, lmax, ks, etas, pools, p, steps, rows, iters)
    agree = []
    for q, k in enumerate(ks):
        for j in range(J):
            exact = _traj_agree(res["traj"][q, j], ref["traj"][q][j], k)
            if exact:
                assert res["lambda_k"][q, j] == ref["lambda_k"][q][j]
            agree.append(oracle.ari(res["labels"][q, j], ref["labels"][q][j]))
    # float32 features against float64: a few boundary points may move
    assert np.mean(agree) >= 0.995 and np.min(agree) >= 0.97, agree
    assert np.max(np.abs(res["gamma"] - ref["gamma"])) <= 0.03
    # gamma from the returned labels, recomputed by the oracle's ARI
    for q in range(len(ks)):
        assert res["gamma"][q] == pytest.approx(oracle.gamma(list(res["labels"][q])), rel=1e-12)
    assert np.all(res["inertia"] > 0)


def test_stability_bfloat16_signals_and_single_k():
    g = W.cliques(4, 16, bridges=True)
    ks = [4]
    J, reps, p, steps, iters = 3, 2, 50, 10, 8
    eta_max = 8
    Rs, _ = W.stability_pools(g.n, J, eta_max, 31)
    Rb = W.bf16_round(Rs)
    rows = W.stability_init_rows(g.n, ks, J, reps, 32)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, None)
    lmax = 1.01 * oracle.lambda_max_exact(L)
    G = upload_graph(g)
    out = asc.stability(G, scalar(lmax), 4, 4, [8], J, reps, p, steps, iters, block_bf16(Rb), eta_max, to_dev(rows))
    assert host(out["gamma"])[0] == 1.0
    for j in range(J):
        assert oracle.ari(host(out["labels"])[0, j], g.labels) == 1.0


def test_stability_full_benchmark_size_sampled():
    # the benchmarked sweep (5000-point planar mixture, k = 2..20, J = 20,
    # 20 replicates, p = 150) in one call; the oracle recomputes sampled
    # (k, realisation) cells one by one
    import workloads as W2
    c = 6
    cfg = W2.WORKLOADS[c]
    g, ks, etas, J, (Rs, _), rows = W2.stability_workload(c)
    eta_max = max(etas)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, None)
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, None)
    lmax = oracle.lmax_estimate(L, s, W2.start_vector(g.n, W2.workload_seeds(c)["lanczos"]), 60)
    G = upload_graph(g)
    out = asc.stability(G, scalar(lmax), ks[0], ks[-1], etas, J, cfg["reps"], cfg["p"], cfg["steps"],
                        cfg["kmeans_iters"], block_f32(Rs), eta_max, to_dev(rows))
    res = {k_: host(v) for k_, v in out.items()}
    pools = _pools(Rs, J, eta_max)
    assert np.all(np.abs(res["gamma"]) <= 1.0)
    for q in range(len(ks)):
        assert res["gamma"][q] == pytest.approx(np.mean(res["ari"][q]), rel=1e-12)
    agree = []
    for q, j in [(0, 3), (8, 0), (9, 11), (18, 19)]:
        k = ks[q]
        F, est, traj = oracle.features(L, lmax, k, etas[q], pools[j], cfg["p"], cfg["steps"])
        if _traj_agree(res["traj"][q, j], traj, k):
            assert res["lambda_k"][q, j] == est
        lab, best, ins = oracle.kmeans_replicates(F, k, rows[q, j], cfg["kmeans_iters"])
        # the chosen replicate's inertia is the oracle's least one
        assert np.min(res["inertia"][q, j]) == pytest.approx(np.min(ins), rel=1e-4)
        agree.append(oracle.ari(res["labels"][q, j], lab))
    assert np.mean(agree) >= 0.97, agree


def test_features_of_every_k_at_once_equal_one_k_at_a_time():
    # up to 32 values of k the sweep forms every k's features in one pass over
    # the state store, above that one k at a time; on the same signals (same
    # eta_max, so the same realisations) and initial rows the overlapping k
    # must give bit-identical estimates, labels and gamma
    x, _ = W.gmm2d_points(1000, 5, 91)
    g = W.knn_graph(x, int(round(np.log(1000))))
    J, reps, p, steps, iters, eta_max = 3, 2, 40, 8, 5, 72
    Rs, _ = W.stability_pools(g.n, J, eta_max, 41)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, None)
    lmax = 1.01 * oracle.lambda_max_exact(L)
    G = upload_graph(g)
    out = {}
    for ks in (list(range(2, 37)), list(range(2, 21))):
        rows = W.stability_init_rows(g.n, ks, J, reps, 42)
        res = asc.stability(G, scalar(lmax), ks[0], ks[-1], [2 * k for k in ks], J, reps, p, steps, iters,
                            block_f32(Rs), eta_max, to_dev(rows))
        out[len(ks)] = {k_: host(v) for k_, v in res.items()}
    per_k, all_k = out[35], out[19]
    np.testing.assert_array_equal(per_k["lambda_k"][:19], all_k["lambda_k"])
    np.testing.assert_array_equal(per_k["labels"][:19], all_k["labels"])
    np.testing.assert_array_equal(per_k["inertia"][:19], all_k["inertia"])
    np.testing.assert_array_equal(per_k["gamma"][:19], all_k["gamma"])
