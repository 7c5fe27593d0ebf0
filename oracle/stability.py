"""Stability measure gamma(k) for choosing the number of clusters (Sec. 4.3,
Eq. stab) and the adjusted Rand index it averages (Hubert & Arabie, J.
Classification 1985).  Test infrastructure only.

Readings taken here:
  * gamma(k) is the mean ARI over the J(J-1)/2 unordered pairs of the J
    clusterings (the printed double sum runs over i != j with the weight
    2/(J(J-1)), which would count every pair twice; the text calls it the mean
    over all pairs, so each unordered pair counts once);
  * realisation j for a given k draws its eta_k signals as the first eta_k
    columns of the j-th pool of unit-variance Gaussian columns, scaled by
    1/sqrt(eta_k) (variance 1/eta, Sec. 3.1); realisations are independent
    for a fixed k;
  * every realisation runs the whole algorithm (Sec. 4.1 steps 2-6): lambda_k
    by the dichotomy on its own signals, the filter at that cut-off, row
    normalisation, and k-means: Lloyd for a fixed number of iterations from
    each of `reps` sets of k initial rows (replicates, Sec. 5), keeping the
    replicate of least inertia sum_i min_c |f_i - mu_c|^2 (float64; the lowest
    replicate index on ties).  Initial rows are drawn uniformly without
    replacement and passed in (the k-means++ seeding of the paper's software
    is not reproduced);
  * the ARI of two partitions whose index denominator vanishes (both one
    cluster, or both all singletons) is 1.

Pinned by (tests/test_oracle_stability.py): exact rational ARI from the pair
counts of every pair of points (brute force) on small inputs, scikit-learn's
adjusted_rand_score, invariance under relabelling and symmetry, the special
cases; gamma = 1 at the number of disjoint cliques of a graph and < 1 away from
it (the detection property the paper reports for its Fig. 2 experiment).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from .cheb import cheb_coeffs, cheb_filter
from .cluster import kmeans_lloyd, normalize_rows
from .eigcount import dichotomy_moments


def contingency(a, b):
    """n_uv = #{i : a_i = u, b_i = v} as exact Python integers (dict)."""
    tab = {}
    for u, v in zip(np.asarray(a).tolist(), np.asarray(b).tolist()):
        tab[(u, v)] = tab.get((u, v), 0) + 1
    return tab


def _c2(x: int) -> int:
    return x * (x - 1) // 2


def ari_terms(a, b):
    """(index, sum_u C(a_u,2), sum_v C(b_v,2), C(n,2)) as exact integers."""
    tab = contingency(a, b)
    rows, cols = {}, {}
    index = 0
    for (u, v), m in tab.items():
        index += _c2(m)
        rows[u] = rows.get(u, 0) + m
        cols[v] = cols.get(v, 0) + m
    sa = sum(_c2(m) for m in rows.values())
    sb = sum(_c2(m) for m in cols.values())
    return index, sa, sb, _c2(len(np.asarray(a)))


def ari(a, b) -> float:
    """ARI = (index - E[index]) / (max index - E[index]) with
    E[index] = sa sb / C(n,2) and max index = (sa + sb)/2."""
    index, sa, sb, n2 = ari_terms(a, b)
    if n2 == 0:
        return 1.0
    expected = Fraction(sa * sb, n2)
    mx = Fraction(sa + sb, 2)
    if mx == expected:
        return 1.0
    return float((index - expected) / (mx - expected))


def ari_pairs(labels):
    """ARIs of the clusterings labels[0..J-1] over the pairs (i, j), i < j,
    in the order (0,1), (0,2), ..., (0,J-1), (1,2), ..."""
    J = len(labels)
    return np.array([ari(labels[i], labels[j]) for i in range(J) for j in range(i + 1, J)])


def gamma(labels) -> float:
    """Mean ARI over all unordered pairs (Eq. stab)."""
    return float(np.mean(ari_pairs(labels)))


def realisation_signals(pool, eta):
    """The first eta unit-variance columns, scaled to variance 1/eta."""
    return np.asarray(pool, dtype=np.float64)[:, :eta] / np.sqrt(eta)


def inertia(F, C, labels) -> float:
    """sum_i |f_i - mu_{label_i}|^2 in float64 (squares rounded before the adds)."""
    F = np.asarray(F, dtype=np.float64)
    D = F - np.asarray(C, dtype=np.float64)[np.asarray(labels)]
    return float(np.sum(np.sum(D * D, axis=1)))


def kmeans_replicates(F, k, init_rows, iters):
    """Lloyd from each replicate's initial rows init_rows[rep][:k]; returns
    (labels of the least-inertia replicate, its index, all inertias)."""
    best, best_rep, all_in = None, -1, []
    for rep, rows in enumerate(init_rows):
        labels, C = kmeans_lloyd(F, F[np.asarray(rows)[:k]], iters)
        e = inertia(F, C, labels)
        all_in.append(e)
        if best is None or e < all_in[best_rep]:
            best, best_rep = labels, rep
    return best, best_rep, np.array(all_in)


def features(L, lmax, k, eta, pool, p, steps):
    """Steps 2-5 for one realisation: (normalised features, lambda_k estimate, trajectory)."""
    R = realisation_signals(pool, eta)
    est, traj = dichotomy_moments(L, lmax, k, p, steps, R)
    Y = cheb_filter(L, lmax, cheb_coeffs(est, lmax, p), R)
    F, _ = normalize_rows(Y)
    return F, est, traj


def cluster_once(L, lmax, k, eta, pool, p, steps, init_rows, iters):
    """One run of the algorithm for k clusters on one realisation; init_rows
    is [reps][>= k].  Returns (labels, lambda_k estimate, trajectory)."""
    F, est, traj = features(L, lmax, k, eta, pool, p, steps)
    labels, _, _ = kmeans_replicates(F, k, init_rows, iters)
    return labels, est, traj


def stability(L, lmax, ks, etas, pools, p, steps, init_rows, iters):
    """gamma(k) for every k in ks.  pools[j] is realisation j's n x eta_max
    unit-variance block; init_rows[q][j][rep] the initial centroid rows (first
    k used) of replicate rep for ks[q].  Returns dict with gamma[q],
    ari[q][pair], labels[q][j], lambda_k[q][j], traj[q][j]."""
    out = {"gamma": [], "ari": [], "labels": [], "lambda_k": [], "traj": []}
    for q, (k, eta) in enumerate(zip(ks, etas)):
        labs, lams, trs = [], [], []
        for j, pool in enumerate(pools):
            lab, est, traj = cluster_once(L, lmax, k, eta, pool, p, steps, init_rows[q][j], iters)
            labs.append(lab)
            lams.append(est)
            trs.append(traj)
        a = ari_pairs(labs)
        out["gamma"].append(float(np.mean(a)))
        out["ari"].append(a)
        out["labels"].append(labs)
        out["lambda_k"].append(lams)
        out["traj"].append(trs)
    out["gamma"] = np.array(out["gamma"])
    return out
