"""The algorithmic byte counts behind the bench line's roofline objects
(host arithmetic only): the per-step formulas against the figures of the
method's accounting for the benchmark configurations, and the counter-traffic
lookup that goes null when the measured kernel source changes."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_step_bytes_of_the_configurations():
    # B_step = row_ptr + col/w + diagonal + T_j, T_{j-1}, T_{j+1} + Y read and write
    n, nnz = 1_000_000, 30_000_000
    assert bench.b_step(n, nnz, 96, 4) == 4 * (n + 1) + 8 * nnz + 4 * n + 3 * n * 96 * 4 + 2 * n * 96 * 4
    assert bench.b_step(n, nnz, 96, 4) / 1e6 == pytest.approx(2168, rel=1e-3)       # float32 states
    assert bench.b_step(n, nnz, 96, 2) / 1e6 == pytest.approx(1592, rel=1e-3)       # bfloat16 states
    assert bench.b_step(100_000, 2_000_000, 64, 4) / 1e6 == pytest.approx(145, rel=1e-2)
    # pattern-only graphs stream no weights
    assert bench.b_step(n, nnz, 96, 4) - bench.b_step(n, nnz, 96, 4, weighted=False) == 4 * nnz


def test_adjoint_step_bytes():
    # B_mat + n r (4 b + 4) + 8 nnz: A_{j+1}, A_{j+2}, A_j, T_j in state precision,
    # G in float32, the per-entry accumulator read and written
    n, nnz, r = 1_000_000, 30_000_000, 96
    b_mat = 4 * (n + 1) + 8 * nnz + 4 * n
    assert bench.b_adj_step(n, nnz, r, 4) == b_mat + n * r * 20 + 8 * nnz
    assert bench.b_adj_step(n, nnz, r, 4) / 3 / 1e9 == pytest.approx(0.80, abs=0.01)  # per 32-column slice


def test_counter_traffic_goes_null_when_the_kernel_changes(monkeypatch):
    wl = bench.STEP_TRAFFIC["workload"]
    t = bench.step_traffic_bytes(wl, 32, 4)
    if bench.step_kernel_sha1() == bench.STEP_TRAFFIC["src_sha1"]:
        kib = bench.STEP_TRAFFIC["kib_per_launch"][(32, 4)]
        assert t == pytest.approx(1024 * (2.0 * kib[0] + 1.0 * kib[1]))
    monkeypatch.setattr(bench, "step_kernel_sha1", lambda: "0" * 40)
    assert bench.step_traffic_bytes(wl, 32, 4) is None
    assert bench.step_traffic_bytes("another workload", 32, 4) is None
    monkeypatch.setattr(bench, "adj_kernel_sha1", lambda: "0" * 40)
    assert bench.adj_traffic_bytes(wl, 32, 4) is None


def test_committed_counter_figures_match_the_committed_kernels():
    # the stored counter bytes were taken on the kernels of this tree
    assert bench.step_kernel_sha1() == bench.STEP_TRAFFIC["src_sha1"]
    assert bench.step_kernel_sha1() == bench.BLOCK_STEP_TRAFFIC["src_sha1"]
    assert bench.adj_kernel_sha1() == bench.ADJ_TRAFFIC["src_sha1"]
