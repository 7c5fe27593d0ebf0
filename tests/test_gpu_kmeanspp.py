"""GPU parity of the k-means++ seeding (exact integer D^2 draw) against the
oracle: the chosen rows are compared exactly."""
import numpy as np
import pytest
import torch

from oracle import kmeanspp as kpp
import workloads as W
import paper_1509_08863_amd as asc

from gpu_util import DEV, block_f32, host

pytestmark = pytest.mark.gpu


def _u(k, seed):
    return torch.from_numpy(W.seeding_draws(k, seed).astype(np.int64)).to(DEV)


@pytest.mark.parametrize("n,r,k", [(1000, 8, 10), (4099, 33, 64), (300_001, 16, 20), (257, 3, 257), (5, 2, 1),
                                   (2049, 40, 30), (1500, 100, 50), (70, 64, 64)])
def test_kmeanspp_rows_match_oracle(n, r, k):
    rng = np.random.default_rng(n + k)
    F = rng.standard_normal((n, r)).astype(np.float32)
    U = W.seeding_draws(k, n)
    rows = host(asc.kmeans_pp(block_f32(F), k, torch.from_numpy(U.astype(np.int64)).to(DEV)))
    np.testing.assert_array_equal(rows, kpp.kmeans_pp_rows(F, k, U))
    if k == n:
        assert sorted(rows.tolist()) == list(range(n))


def test_kmeanspp_duplicates_and_coincident_rows():
    # clusters of exact copies: chosen rows never repeat a copy set while a
    # distinct one remains; then every weight is 0 and the uniform index is used
    base = np.random.default_rng(1).standard_normal((4, 6)).astype(np.float32)
    F = np.repeat(base, 25, axis=0)
    U = W.seeding_draws(7, 2)
    rows = host(asc.kmeans_pp(block_f32(F), 7, torch.from_numpy(U.astype(np.int64)).to(DEV)))
    ref = kpp.kmeans_pp_rows(F, 7, U)
    np.testing.assert_array_equal(rows, ref)
    assert len({r // 25 for r in rows[:4]}) == 4


def test_kmeanspp_draws_are_taken_modulo_2_53():
    F = np.random.default_rng(5).standard_normal((3000, 12)).astype(np.float32)
    U = W.seeding_draws(9, 6).astype(np.int64)
    a = host(asc.kmeans_pp(block_f32(F), 9, torch.from_numpy(U).to(DEV)))
    b = host(asc.kmeans_pp(block_f32(F), 9, torch.from_numpy(U | (np.int64(1) << 60)).to(DEV)))
    np.testing.assert_array_equal(a, b)


def test_kmeanspp_full_size_features():
    # the 1e6-row, 96-column feature shape of the pipeline, k = 12 draws
    rng = np.random.default_rng(11)
    F = rng.standard_normal((1_000_000, 96)).astype(np.float32)
    F /= np.linalg.norm(F, axis=1, keepdims=True)
    U = W.seeding_draws(12, 13)
    rows = host(asc.kmeans_pp(block_f32(F), 12, torch.from_numpy(U.astype(np.int64)).to(DEV)))
    np.testing.assert_array_equal(rows, kpp.kmeans_pp_rows(F, 12, U))
