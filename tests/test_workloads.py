"""The seeded generators produce the graphs they describe."""
import numpy as np
import scipy.sparse as sp

import workloads as W


def _check_csr(g):
    rp = g.row_ptr.astype(np.int64)
    ci = g.col_idx.astype(np.int64)
    assert rp[0] == 0 and rp[-1] == g.nnz and np.all(np.diff(rp) >= 0)
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    assert not np.any(rows == ci)
    same = rows[1:] == rows[:-1]
    assert np.all(ci[1:][same] > ci[:-1][same])
    A = sp.csr_matrix((np.ones(g.nnz), ci, rp), shape=(g.n, g.n))
    assert (A - A.T).nnz == 0


def test_sbm_c1_shape_and_determinism():
    g = W.workload_graph(1)
    _check_csr(g)
    assert g.n == 1000
    assert 14 < g.nnz / g.n < 18           # mean degree 16
    h = W.workload_graph(1)
    assert np.array_equal(g.col_idx, h.col_idx)
    # intra-community edges dominate: eps = 0.1 -> p_out/p_in = 0.1
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    intra = np.mean(g.labels[rows] == g.labels[g.col_idx])
    expected = 99 / (99 + 0.1 * 900)
    assert abs(intra - expected) < 0.05


def test_sbm_dirichlet_sizes_sum():
    s = W.dirichlet_sizes(10000, 50, 5.0, 3)
    assert s.sum() == 10000 and len(s) == 50


def test_gmm_knn_graph():
    g = W.gmm_knn(2000, 16, 20, 10, 5)
    _check_csr(g)
    deg = np.diff(g.row_ptr)
    assert deg.min() >= 10 and 10 <= deg.mean() <= 20
    assert np.all(g.d2 > 0)
    # the squared lengths are symmetric
    A = sp.csr_matrix((g.d2.astype(np.float64), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    assert abs(A - A.T).max() == 0


def test_signals_variance_and_bf16():
    x, x64 = W.signals(4000, 64, 1)
    assert x.dtype == np.float32
    assert abs(x64.var() * 64 - 1) < 0.02
    b, b64 = W.signals(100, 8, 1, "bf16")
    assert b.dtype == np.uint16
    f = W.signals(100, 8, 1)[0]
    assert np.max(np.abs(b64 - f) / np.abs(f)) <= 2.0 ** -8
    # round to nearest even on exact ties
    t = np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8], dtype=np.float32)
    np.testing.assert_array_equal(W.bf16_to_f32(W.bf16_round(t)), [1.0, 1.0 + 2 ** -6])


def test_named_graphs():
    for g in (W.complete(5), W.cycle(7), W.path(4), W.star(6), W.cliques(3, 4, True),
              W.random_weighted(20, 0.3, 1, isolated=2)):
        _check_csr(g)


def test_locality_order_is_a_relabelling():
    import oracle
    g = W.gmm_knn(1500, 16, 5, 10, 3)
    h, perm = W.locality_order(g)
    _check_csr(h)
    assert sorted(perm.tolist()) == list(range(g.n))
    w_g = oracle.gauss_weights(g.d2.astype(np.float64), 2.0)
    w_h = oracle.gauss_weights(h.d2.astype(np.float64), 2.0)
    Lg = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, w_g)
    Lh = oracle.laplacian_sparse(h.n, h.row_ptr, h.col_idx, w_h)
    assert abs(Lg[perm][:, perm] - Lh).max() <= 1e-12  # strengths summed in another order
    # the filter commutes with the relabelling
    R = W.signals_f64(g.n, 4, 2)
    a = oracle.cheb_coeffs(1.0, 20.0, 30)
    np.testing.assert_allclose(oracle.cheb_filter(Lh, 20.0, a, R[perm]), oracle.cheb_filter(Lg, 20.0, a, R)[perm],
                               rtol=1e-12, atol=1e-14)
    # neighbours end up closer in index space
    rows_g = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    rows_h = np.repeat(np.arange(h.n), np.diff(h.row_ptr))
    assert np.abs(rows_h - h.col_idx).mean() < 0.5 * np.abs(rows_g - g.col_idx).mean()


def test_block_order_makes_blocks_contiguous():
    import oracle
    g = W.sbm(W.dirichlet_sizes(3000, 6, 5.0, 4), 12.0, 0.05, 5)
    h, perm = W.block_order(g)
    _check_csr(h)
    assert sorted(perm.tolist()) == list(range(g.n))
    # labels non-decreasing, every block one contiguous range
    assert np.all(np.diff(h.labels) >= 0)
    np.testing.assert_array_equal(h.labels, g.labels[perm])
    Lg = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, None)
    Lh = oracle.laplacian_sparse(h.n, h.row_ptr, h.col_idx, None)
    assert abs(Lg[perm][:, perm] - Lh).max() == 0.0
    # intra-block edges now join nearby indices: most stored entries stay in the row's block
    rows = np.repeat(np.arange(h.n), np.diff(h.row_ptr))
    assert np.mean(h.labels[rows] == h.labels[h.col_idx]) > 0.5
