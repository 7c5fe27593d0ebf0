"""Pins of the k-means++ seeding oracle (D^2 draw with integer weights)."""
import numpy as np
import pytest

from oracle import kmeanspp as kpp
import workloads as W

TOP = (1 << 53) - 1


def test_distances_by_hand():
    F = np.array([[0, 0], [3, 4], [6, 8], [-1, 0]], dtype=np.float32)
    np.testing.assert_array_equal(kpp.sqdist_to_row(F.astype(np.float64), np.array([0.0, 0.0])), [0, 25, 100, 1])
    np.testing.assert_array_equal(kpp.weights(np.array([0.0, 25.0, 100.0, 1.0])),
                                  [0, (1 << 30) // 4, 1 << 30, (1 << 30) // 100])


def test_second_pick_follows_the_squared_distance():
    # rows 0, 1, 3 on a line, first pick row 0 (U_0 = 0): D = (0, 1, 9), so
    # row 1 comes second with probability 1/10 (the D law would give 1/4)
    F = np.array([[0.0], [1.0], [3.0]], dtype=np.float32)
    U = W.seeding_draws(20000, 7)
    ones = sum(int(kpp.kmeans_pp_rows(F, 2, [0, int(u)])[1] == 1) for u in U)
    freq = ones / len(U)
    q1, q2 = (1 << 30) // 9, 1 << 30
    p = q1 / (q1 + q2)
    assert abs(p - 0.1) < 1e-8
    assert abs(freq - p) < 4 * np.sqrt(p * (1 - p) / len(U))


def test_integer_mapping_at_the_ends():
    F = np.array([[0.0], [2.0], [5.0], [5.0], [9.0]], dtype=np.float32)
    # U_0 = 0 -> row 0; U_0 = 2^53 - 1 -> row n - 1
    assert kpp.kmeans_pp_rows(F, 1, [0])[0] == 0
    assert kpp.kmeans_pp_rows(F, 1, [TOP])[0] == 4
    # after row 0, U = 0 takes the first row of positive weight, U = 2^53 - 1 the last
    assert kpp.kmeans_pp_rows(F, 2, [0, 0])[1] == 1
    assert kpp.kmeans_pp_rows(F, 2, [0, TOP])[1] == 4


def test_all_rows_when_k_equals_n():
    rng = np.random.default_rng(3)
    F = rng.standard_normal((12, 3)).astype(np.float32)
    rows = kpp.kmeans_pp_rows(F, 12, W.seeding_draws(12, 5))
    assert sorted(rows.tolist()) == list(range(12))


def test_the_only_distinct_row_comes_second():
    F = np.zeros((50, 4), dtype=np.float32)
    F[37] = 1.0
    for u in W.seeding_draws(20, 9):
        rows = kpp.kmeans_pp_rows(F, 2, [int(u), int(u)])
        assert rows[1] == (37 if rows[0] != 37 else rows[1])
        if rows[0] != 37:
            assert rows[1] == 37


def test_all_coincident_rows_fall_back_to_the_uniform_index():
    F = np.ones((10, 2), dtype=np.float32)
    rows = kpp.kmeans_pp_rows(F, 3, [0, TOP, 1 << 52])
    assert rows.tolist() == [0, 9, 5]


def test_rejects_bad_draws():
    F = np.ones((4, 2), dtype=np.float32)
    with pytest.raises(ValueError):
        kpp.kmeans_pp_rows(F, 5, [0] * 5)
    with pytest.raises(ValueError):
        kpp.kmeans_pp_rows(F, 2, [0, 1 << 53])
