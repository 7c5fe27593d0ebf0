"""GPU parity of k-means with replicates (Sec. 5 clusters with k-means and 20
replicates): every run of the batched entry point against the same run made
of the single-problem assignment and update calls (which take every step),
bit for bit, and against the FP64 oracle's replicates."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_1509_08863_amd as asc

from gpu_util import DEV, host, to_dev

pytestmark = pytest.mark.gpu


def _data(n, r, k, reps, seed):
    # overlapping clusters (component spread comparable to the mean spread),
    # so that the runs need different numbers of steps to settle
    x, _ = W.gmm_points(n, r, max(k, 2), seed, comp_sigma=1.0, mean_sigma=1.5)
    rng = np.random.default_rng(seed + 1)
    rows = np.stack([rng.choice(n, size=k, replace=False) for _ in range(reps)]).astype(np.int32)
    return x.astype(np.float32), rows


def _step_by_step(F, rows_q, iters):
    """One run through the single-problem calls, every step taken; returns
    (labels, C, the last step whose assignment moved a label)."""
    C = asc.kmeans_init_rows(F, to_dev(rows_q))
    prev, last = None, -1
    for it in range(iters):
        lab, _ = asc.kmeans_assign(F, C, dist=False)
        if prev is not None and not torch.equal(lab, prev):
            last = it
        prev = lab
        asc.kmeans_update(F, lab, C)
    lab, _ = asc.kmeans_assign(F, C)
    return host(lab), host(C), last


# shapes that reach every assignment kernel (matrix cores with staged and with
# loaded rows, one lane per centroid with several rows per pass, the grouped
# and the plain kernel) and every centroid-sum kernel (slots, four copies, one
# copy, sums in global memory; final sums by lanes and by wavefronts)
CASES = [
    (3000, 8, 8, 12, 25),
    (2049, 40, 5, 6, 15),
    (1500, 16, 40, 4, 12),
    (1000, 40, 100, 3, 8),
    (700, 64, 200, 2, 6),
    (10000, 6, 3, 5, 20),
    (6000, 8, 6, 3, 10),  # 24 partial blocks, cut to 16 on both paths
    (500, 4, 1, 3, 5),
    (800, 8, 6, 4, 0),
    (333, 3, 4, 1, 10),
]


@pytest.mark.parametrize("n,r,k,reps,iters", CASES)
def test_replicates_equal_the_step_by_step_runs(n, r, k, reps, iters):
    x, rows = _data(n, r, k, reps, 7000 + n + k)
    F = to_dev(x)
    lab, C, inertia = asc.kmeans_replicates(F, to_dev(rows), iters)
    lab, C, inertia = host(lab), host(C), host(inertia)
    runs = [_step_by_step(F, rows[q], iters) for q in range(reps)]
    # every run's inertia is that of its own final labels and centroids
    want = np.array([oracle.inertia(x, Cq, lq) for lq, Cq, _ in runs])
    np.testing.assert_allclose(inertia, want, rtol=1e-12, atol=0)
    best = int(np.argmin(inertia))  # the lowest run on ties
    np.testing.assert_array_equal(lab, runs[best][0])
    np.testing.assert_array_equal(C.view(np.uint32), runs[best][1].view(np.uint32))


def test_runs_that_settle_at_different_steps():
    # the runs of the main case settle at different steps, some well before
    # the last, so the skipped steps are really exercised; each run's final
    # labels and centroids (through its inertia) are still the full run's
    n, r, k, reps, iters = 3000, 8, 8, 12, 25
    x, rows = _data(n, r, k, reps, 7000 + n + k)
    F = to_dev(x)
    lasts = [_step_by_step(F, rows[q], iters)[2] for q in range(reps)]
    assert min(lasts) < iters // 2 and len(set(lasts)) >= 3, lasts


def test_replicates_match_the_oracle():
    n, r, k, reps, iters = 3000, 8, 8, 12, 25
    x, rows = _data(n, r, k, reps, 7000 + n + k)
    lab, C, inertia = asc.kmeans_replicates(to_dev(x), to_dev(rows), iters)
    ref_lab, ref_best, ref_in = oracle.kmeans_replicates(x, k, rows, iters)
    np.testing.assert_allclose(host(inertia), ref_in, rtol=1e-12, atol=0)
    np.testing.assert_array_equal(host(lab), ref_lab)


def test_replicates_reject_bad_arguments():
    x, rows = _data(100, 4, 3, 2, 5)
    F = to_dev(x)
    bad = [(np.zeros((2, 0), np.int32), 5), (np.zeros((2, 1025), np.int32), 5), (rows, -1), (rows, 10001),
           (np.zeros((0, 3), np.int32), 5)]
    for rw, iters in bad:
        with pytest.raises(asc.AscError):
            asc.kmeans_replicates(F, to_dev(rw), iters)
