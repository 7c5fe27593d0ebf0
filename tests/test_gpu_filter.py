"""GPU parity of the polynomial filter, coefficients, strengths and lambda_max
against the FP64 oracle (Sec. 2.1, Sec. 2.4, Sec. 3.1, Sec. 4.1 steps 1, 3-5)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_1509_08863_amd as asc

from gpu_util import DEV, upload_graph, block_f32, block_bf16, scalar, host, rel_fro, to_dev

pytestmark = pytest.mark.gpu

# float32 states: relative Frobenius error against float64 (stated requirement)
TOL_F32 = 1e-5
# bfloat16 states, float32 arithmetic: measured error vs float64 on the same
# (bf16-rounded) R is below 3e-2 on these graphs; bound stated with margin
TOL_BF16 = 6e-2


def _oracle_setup(g, r, seed, p, frac=0.17, w=None):
    ww = g.weights_or_ones() if w is None else w
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, ww.astype(np.float64))
    lmax = 1.01 * oracle.lambda_max_exact(L)
    a = oracle.cheb_coeffs(frac * lmax, lmax, p)
    return L, lmax, a


GRAPHS = {
    "sbm_c1": lambda: W.workload_graph(1),
    "weighted_isolated": lambda: W.random_weighted(700, 0.02, 3, isolated=9),
    "path": lambda: W.path(50),
    "single_node_pairs": lambda: W.from_edges(5, [(0, 1)]),
}


def test_strength_matches_oracle():
    g = W.random_weighted(500, 0.05, 1, isolated=3)
    G = upload_graph(g)
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, g.w.astype(np.float64))
    np.testing.assert_allclose(host(G.strength), s, rtol=1e-15, atol=0)


@pytest.mark.parametrize("bad", ["unsorted", "asymmetric", "selfloop", "negative"])
def test_validation_rejects(bad):
    g = W.random_weighted(40, 0.2, 2)
    ci = g.col_idx.copy()
    w = g.w.copy()
    if bad == "unsorted":
        i = int(np.argmax(np.diff(g.row_ptr) >= 2))
        a, b = g.row_ptr[i], g.row_ptr[i] + 1
        ci[a], ci[b] = ci[b], ci[a]
    elif bad == "asymmetric":
        w[0] *= 1.5
    elif bad == "selfloop":
        ci[0] = 0
    elif bad == "negative":
        w[3] = -1.0
    gg = W.Graph(n=g.n, row_ptr=g.row_ptr, col_idx=ci, w=w)
    with pytest.raises(asc.AscError) as e:
        upload_graph(gg, validate=True)
    assert e.value.status == 1
    upload_graph(g, validate=True)  # the valid graph passes


@pytest.mark.parametrize("name", ["sbm_c1", "weighted_isolated", "path"])
@pytest.mark.parametrize("iters", [5, 40])
def test_lmax_matches_oracle_lanczos(name, iters):
    g = GRAPHS[name]()
    G = upload_graph(g)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, g.weights_or_ones().astype(np.float64))
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, g.weights_or_ones().astype(np.float64))
    v0 = W.start_vector(g.n, 5)
    ref = oracle.lmax_estimate(L, s, v0, iters)
    got, got_h = asc.lmax_estimate(G, to_dev(v0), iters, host=True)
    assert got_h == pytest.approx(ref, rel=1e-9)
    lam_n = oracle.lambda_max_exact(L)
    if iters >= 40:
        assert lam_n <= got_h <= 1.0101 * lam_n


def test_coeffs_match_oracle():
    lmax = scalar(37.5)
    lc = to_dev(np.array([-1.0, 0.0, 3.3, 18.75, 30.0, 37.5, 50.0]))
    for p in (0, 1, 7, 150):
        for jack in (True, False):
            got = host(asc.cheb_coeffs(lc, lmax, p, jack))
            for q, x in enumerate([-1.0, 0.0, 3.3, 18.75, 30.0, 37.5, 50.0]):
                ref = oracle.cheb_coeffs(x, 37.5, p, jack)
                np.testing.assert_allclose(got[q], ref, rtol=1e-13, atol=1e-15)


def _run_filter_case(g, r, p, dtype, seed=3, frac=0.17, weighted=True, ld=None):
    w = g.weights_or_ones()
    L, lmax, a = _oracle_setup(g, r, seed, p, frac, w)
    G = upload_graph(g, unit_as_null=not weighted)
    if dtype == "f32":
        Rs, R64 = W.signals(g.n, r, seed)
        Rd = block_f32(Rs, ld)
    else:
        Rs, R64 = W.signals(g.n, r, seed, "bf16")
        Rd = block_bf16(Rs, ld)
    Y = asc.cheb_filter(G, scalar(lmax), to_dev(a), Rd)
    Yref = oracle.cheb_filter(L, lmax, a, R64)
    return host(Y), Yref


@pytest.mark.parametrize("name", ["sbm_c1", "weighted_isolated", "path", "single_node_pairs"])
@pytest.mark.parametrize("r", [1, 3, 8, 32, 48, 97])
@pytest.mark.parametrize("p", [0, 1, 2, 3, 50])
def test_filter_f32_parity(name, r, p):
    g = GRAPHS[name]()
    Y, Yref = _run_filter_case(g, r, p, "f32", weighted=(name != "sbm_c1"))
    assert rel_fro(Y, Yref) <= TOL_F32


@pytest.mark.parametrize("name", ["sbm_c1", "weighted_isolated"])
@pytest.mark.parametrize("r", [3, 16, 64, 96])
@pytest.mark.parametrize("p", [1, 50])
def test_filter_bf16_parity(name, r, p):
    g = GRAPHS[name]()
    Y, Yref = _run_filter_case(g, r, p, "bf16")
    err = rel_fro(Y, Yref)
    print(f"bf16 {name} r={r} p={p} rel_fro={err:.3e}")
    assert err <= TOL_BF16


def test_filter_wide_leading_dimension_and_unit_weights_path():
    g = W.workload_graph(1)
    Y1, Yref = _run_filter_case(g, 20, 40, "f32", weighted=False, ld=40)
    Y2, _ = _run_filter_case(g, 20, 40, "f32", weighted=True, ld=24)
    assert rel_fro(Y1, Yref) <= TOL_F32
    np.testing.assert_array_equal(Y1, Y2)  # w = 1.0 and w = NULL give identical sums


def test_filter_mid_size_sbm():
    g = W.sbm(W.equal_sizes(20000, 20), 20.0, 0.05, 77)
    Y, Yref = _run_filter_case(g, 64, 100, "f32", weighted=False)
    err = rel_fro(Y, Yref)
    print(f"sbm n=2e4 r=64 p=100 rel_fro={err:.3e}")
    assert err <= TOL_F32


def test_all_pass_is_identity():
    # cut-off at lambda_max: a = (1, 0, ..., 0) exactly -> Y = R bit for bit
    g = W.workload_graph(1)
    G = upload_graph(g)
    Rs, _ = W.signals(g.n, 32, 1)
    lmax = scalar(40.0)
    a = asc.cheb_coeffs(scalar(40.0), lmax, 60)
    Y = asc.cheb_filter(G, lmax, a, block_f32(Rs))
    np.testing.assert_array_equal(host(Y), Rs)


def test_constant_vector_gain():
    # L 1 = 0: the constant signal is multiplied by p(-1) = sum_j a_j (-1)^j
    g = W.workload_graph(1)
    G = upload_graph(g)
    lmax = 40.0
    a = oracle.cheb_coeffs(0.17 * lmax, lmax, 100)
    pm1 = float(np.sum(a * (-1.0) ** np.arange(101)))
    Y = host(asc.cheb_filter(G, scalar(lmax), to_dev(a), block_f32(np.ones((g.n, 4)))))
    np.testing.assert_allclose(Y, pm1, rtol=2e-6)


def test_lmax_too_small_is_flagged():
    g = W.workload_graph(1)
    G = upload_graph(g)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, g.weights_or_ones().astype(np.float64))
    lam_n = oracle.lambda_max_exact(L)
    Rs, _ = W.signals(g.n, 8, 1)
    bad = 0.5 * lam_n
    a = to_dev(oracle.cheb_coeffs(0.2 * bad, bad, 40))
    asc.cheb_filter(G, scalar(bad), a, block_f32(Rs))
    with pytest.raises(asc.AscError) as e:
        asc.read_flags(asc.cheb_filter.last_ws)
    assert e.value.status == 5
    asc.cheb_filter(G, scalar(1.01 * lam_n), a, block_f32(Rs))
    assert asc.read_flags(asc.cheb_filter.last_ws) == 0


def test_nan_is_flagged():
    g = W.workload_graph(1)
    G = upload_graph(g)
    Rs, _ = W.signals(g.n, 8, 1)
    Rs[17, 3] = np.nan
    a = to_dev(oracle.cheb_coeffs(5.0, 40.0, 10))
    asc.cheb_filter(G, scalar(40.0), a, block_f32(Rs))
    with pytest.raises(asc.AscError) as e:
        asc.read_flags(asc.cheb_filter.last_ws)
    assert e.value.status == 4


def test_filter_deterministic():
    g = W.workload_graph(1)
    G = upload_graph(g)
    Rs, _ = W.signals(g.n, 32, 2)
    a = to_dev(oracle.cheb_coeffs(5.0, 40.0, 50))
    Y1 = host(asc.cheb_filter(G, scalar(40.0), a, block_f32(Rs)))
    Y2 = host(asc.cheb_filter(G, scalar(40.0), a, block_f32(Rs)))
    np.testing.assert_array_equal(Y1, Y2)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_every_tuned_configuration_is_parity_green(dtype):
    g = W.sbm(W.equal_sizes(6000, 12), 18.0, 0.05, 9)
    r, p = 48, 60
    L, lmax, a = _oracle_setup(g, r, 1, p)
    G = upload_graph(g)
    if dtype == "f32":
        Rs, R64 = W.signals(g.n, r, 4)
        Rd, tdt, widths, tol = block_f32(Rs), torch.float32, (8, 16, 32, 64), TOL_F32
    else:
        Rs, R64 = W.signals(g.n, r, 4, "bf16")
        Rd, tdt, widths, tol = block_bf16(Rs), torch.bfloat16, (16, 32, 64, 128), TOL_BF16
    Yref = oracle.cheb_filter(L, lmax, a, R64)
    try:
        for rs in widths:
            for var in range(8):
                asc.tune_set(G, r, tdt, rs, var)
                assert asc.tune_get(G, r, tdt) == (rs, var)
                Y = host(asc.cheb_filter(G, scalar(lmax), to_dev(a), Rd))
                assert rel_fro(Y, Yref) <= tol, (rs, var)
        rs, var, ms = asc.autotune_filter(G, scalar(lmax), Rd, 2)
        assert rs in widths and 0 <= var <= 7 and ms > 0
        assert asc.tune_get(G, r, tdt) == (rs, var)
        assert rel_fro(host(asc.cheb_filter(G, scalar(lmax), to_dev(a), Rd)), Yref) <= tol
    finally:
        asc.tune_set(G, r, tdt, 0, 0)


def test_tune_table_roundtrip(tmp_path):
    g = W.workload_graph(1)
    G = upload_graph(g)
    asc.tune_set(G, 32, torch.float32, 16, 1)
    path = str(tmp_path / "tune.json")
    asc.tune_save(path)
    asc.tune_set(G, 32, torch.float32, 0, 0)
    assert asc.tune_get(G, 32, torch.float32) == (32, 0)
    asc.tune_load(path)
    assert asc.tune_get(G, 32, torch.float32) == (16, 1)
    asc.tune_set(G, 32, torch.float32, 0, 0)


@pytest.mark.parametrize("n,blocks,weighted", [(300_000, 2, True), (700_000, 3, False)])
def test_lmax_column_blocked_products_match_oracle(n, blocks, weighted):
    # above 2 MB of float64 vector the Lanczos product runs as passes over
    # column ranges (each range L2-resident); the result is the oracle's
    g = W.sbm(W.equal_sizes(n, 4), 8.0, 0.2, 31 + n)
    assert (8 * n + (2 << 20) - 1) // (2 << 20) == blocks
    w = None
    if weighted:  # symmetric weights: a function of the unordered pair
        rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
        cols = g.col_idx.astype(np.int64)
        w = (0.5 + ((rows * cols) % 7) / 7.0).astype(np.float32)
    G = upload_graph(g, w=w) if weighted else upload_graph(g, unit_as_null=True)
    w64 = None if w is None else w.astype(np.float64)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, w64)
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, w64)
    v0 = W.start_vector(g.n, 6)
    ref = oracle.lmax_estimate(L, s, v0, 30)
    _, got = asc.lmax_estimate(G, to_dev(v0), 30, host=True)
    assert got == pytest.approx(ref, rel=1e-9)


@pytest.mark.parametrize("var", [0, 4])
def test_filter_on_block_ordered_graph(var):
    # the same SBM with every generating block contiguous: the filter of the
    # relabelled graph on the relabelled signals is the relabelled filter
    # (each against the float64 oracle of its own graph), on both tile orders
    g = W.sbm(W.dirichlet_sizes(30000, 12, 5.0, 31), 16.0, 0.05, 32)
    h, perm = W.block_order(g)
    r, p = 40, 40
    Rs, R64 = W.signals(g.n, r, 33)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, None)
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, None)
    lmax = oracle.lmax_estimate(L, s, W.start_vector(g.n, 34), 40)
    a = oracle.cheb_coeffs(0.15 * lmax, lmax, p)
    Yo = oracle.cheb_filter(L, lmax, a, R64)
    for graph, R_, ref in ((g, Rs, Yo), (h, Rs[perm], Yo[perm])):
        Gd = upload_graph(graph)
        asc.tune_set(Gd, r, torch.float32, 32, var)
        Y = host(asc.cheb_filter(Gd, scalar(lmax), to_dev(a), block_f32(R_)))
        asc.tune_set(Gd, r, torch.float32, 0, 0)
        assert rel_fro(Y, ref) <= 1e-5
