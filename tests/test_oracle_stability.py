"""Pins of the stability-measure oracle (Sec. 4.3, Eq. stab) and of the
adjusted Rand index (Hubert & Arabie 1985) against facts fixed outside it."""
from fractions import Fraction
from itertools import combinations

import numpy as np
import pytest

import oracle
import workloads as W


def ari_by_pairs(a, b):
    """ARI from the four pair counts over all pairs of points (brute force):
    2(n11 n00 - n10 n01) / ((n11 + n10)(n10 + n00) + (n11 + n01)(n01 + n00))."""
    n11 = n10 = n01 = n00 = 0
    for i, j in combinations(range(len(a)), 2):
        sa, sb = a[i] == a[j], b[i] == b[j]
        if sa and sb:
            n11 += 1
        elif sa:
            n10 += 1
        elif sb:
            n01 += 1
        else:
            n00 += 1
    den = (n11 + n10) * (n10 + n00) + (n11 + n01) * (n01 + n00)
    if den == 0:
        return Fraction(1)
    return Fraction(2 * (n11 * n00 - n10 * n01), den)


@pytest.mark.parametrize("seed", range(12))
def test_ari_equals_pair_count_form_exactly(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 40))
    ka, kb = int(rng.integers(1, 6)), int(rng.integers(1, 6))
    a = rng.integers(0, ka, n)
    b = rng.integers(0, kb, n) if seed % 3 else (a + rng.integers(0, 2, n)) % max(kb, 1)
    assert oracle.ari(a, b) == float(ari_by_pairs(a.tolist(), b.tolist()))


def test_ari_worked_example():
    # pairs together in a: 6, in b: 3, in both: 2, of C(6,2) = 15 -> 8/33
    assert oracle.ari([0, 0, 0, 1, 1, 1], [0, 0, 1, 1, 2, 2]) == 8 / 33


def test_ari_matches_scikit_learn():
    from sklearn.metrics import adjusted_rand_score
    rng = np.random.default_rng(7)
    for n, ka, kb in [(2000, 10, 12), (500, 3, 3), (1000, 50, 2), (300, 1, 7)]:
        a = rng.integers(0, ka, n)
        b = np.where(rng.random(n) < 0.7, a % kb, rng.integers(0, kb, n))
        assert oracle.ari(a, b) == pytest.approx(adjusted_rand_score(a, b), rel=1e-12, abs=1e-14)


def test_ari_invariances_and_special_cases():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 6, 400)
    b = rng.integers(0, 4, 400)
    perm = rng.permutation(6)
    assert oracle.ari(a, b) == oracle.ari(perm[a], b)
    assert oracle.ari(a, b) == oracle.ari(b, a)
    assert oracle.ari(a, a) == 1.0
    assert oracle.ari(perm[a], a) == 1.0
    n = 50
    one, single = np.zeros(n, int), np.arange(n)
    assert oracle.ari(one, one) == 1.0
    assert oracle.ari(single, single) == 1.0
    assert oracle.ari(one, single) == 0.0
    # independent random labellings: ARI near 0 (expectation 0 under permutation)
    vals = [oracle.ari(rng.integers(0, 5, 3000), rng.integers(0, 5, 3000)) for _ in range(20)]
    assert abs(np.mean(vals)) < 2e-3


def test_gamma_is_mean_over_unordered_pairs():
    rng = np.random.default_rng(1)
    A = rng.integers(0, 3, 200)
    B = rng.integers(0, 3, 200)
    v = oracle.ari(A, B)
    assert oracle.gamma([A, B]) == v
    assert oracle.gamma([A, A, B]) == pytest.approx((1.0 + 2 * v) / 3, rel=1e-15)
    np.testing.assert_array_equal(oracle.ari_pairs([A, A, B]), [1.0, v, v])


def test_realisation_scaling_gives_the_eigenvalue_count():
    # with variance 1/eta, <R, p(L) R> estimates the number of eigenvalues below
    # the cut-off; a missing or doubled 1/sqrt(eta) is off by a factor eta or more
    g = W.cliques(6, 12, bridges=True)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, None)
    lmax = 1.01 * oracle.lambda_max_exact(L)
    pool = W.unit_signals(g.n, 600, 5)[1]
    R = oracle.realisation_signals(pool, 600)
    lam = np.linalg.eigvalsh(L.toarray())
    lc = 0.5 * (lam[5] + lam[6])
    c = oracle.eigcount_from_moments(oracle.moments(L, lmax, 120, R), lc, lmax)
    assert abs(c - 6) < 0.6


def test_replicates_keep_least_inertia():
    # four tight groups; replicate 0 starts with two rows in one group (a
    # local optimum), replicate 1 with one row per group (the optimum)
    rng = np.random.default_rng(2)
    centres = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0]], float)
    F = np.repeat(centres, 25, axis=0) + 0.01 * rng.standard_normal((100, 3))
    bad = [0, 1, 30, 60]
    good = [0, 30, 60, 90]
    labels, rep, ins = oracle.kmeans_replicates(F, 4, [bad, good], 10)
    assert rep == 1 and ins[1] < ins[0]
    assert oracle.ari(labels, np.repeat(np.arange(4), 25)) == 1.0
    labels0, rep0, _ = oracle.kmeans_replicates(F, 4, [good, good], 10)
    assert rep0 == 0  # ties keep the lowest replicate


def test_inertia_worked_example_and_lloyd_never_raises_it():
    # by hand: rows (0,0) and (2,0) around (1,0) add 1 + 1, row (5,5) sits on
    # its centroid and (5,7) is 2 above it: 1 + 1 + 0 + 4 = 6
    F = np.array([[0, 0], [2, 0], [5, 5], [5, 7]], float)
    assert oracle.inertia(F, np.array([[1, 0], [5, 5]], float), [0, 0, 1, 1]) == 6.0
    # each Lloyd step (float64 centroids) lowers the inertia or keeps it
    rng = np.random.default_rng(4)
    F = rng.standard_normal((300, 3)) + np.repeat(rng.standard_normal((5, 3)) * 2, 60, axis=0)
    C0 = F[rng.choice(300, 5, replace=False)]
    prev = np.inf
    for it in range(8):
        labels, C = oracle.kmeans_lloyd(F, C0, it, np.float64)
        e = oracle.inertia(F, C, labels)
        assert e <= prev * (1 + 1e-12), (it, e, prev)
        prev = e


def test_gamma_peaks_at_the_number_of_cliques():
    # the detection property of Sec. 4.3: disjoint cliques (one bridge between
    # consecutive ones) are found identically by every realisation at k = 5
    g = W.cliques(5, 20, bridges=True)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, None)
    lmax = 1.01 * oracle.lambda_max_exact(L)
    ks = [3, 4, 5, 6, 7]
    etas = [2 * k for k in ks]
    J, reps = 5, 5
    pools = W.stability_pools(g.n, J, max(etas), 11)[1]
    pools = [pools[:, j * max(etas):(j + 1) * max(etas)] for j in range(J)]
    rows = W.stability_init_rows(g.n, ks, J, reps, 12)
    out = oracle.stability(L, lmax, ks, etas, pools, 60, 12, rows, 10)
    gam = out["gamma"]
    assert gam[2] == 1.0
    assert int(np.argmax(gam)) == 2
    assert all(gam[q] < 1.0 for q in (0, 1, 3, 4))
    for lab in out["labels"][2]:
        assert oracle.ari(lab, g.labels) == 1.0
    for q, k in enumerate(ks):
        assert all(len(np.unique(lab)) <= k for lab in out["labels"][q])
