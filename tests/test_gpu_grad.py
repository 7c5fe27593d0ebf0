"""GPU parity of the gradients (adjoint of the recurrence, Gaussian-kernel
weights, row-normalised loss) against the FP64 oracle, whose gradients are
pinned by finite differences and the Daleckii-Krein formula."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_1509_08863_amd as asc
from paper_1509_08863_amd.autograd import ChebFilter, GaussWeights, RowNormLoss

from gpu_util import DEV, upload_graph, block_f32, block_bf16, scalar, host, rel_fro, to_dev

pytestmark = pytest.mark.gpu

TOL_DW = 1e-4      # float32 states and accumulation, relative Frobenius
TOL_DA = 1e-5      # float64 reductions of float32 products
TOL_DSIGMA = 1e-4


def _problem(n=2000, r=16, p=30, sigma=2.0, seed=5, knn=10):
    g = W.gmm_knn(n, 16, 5, knn, seed)
    d2 = g.d2.astype(np.float64)
    w64 = oracle.gauss_weights(g.d2.astype(np.float32).astype(np.float64), sigma)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, w64)
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, w64)
    lmax = oracle.lmax_estimate(L, s, W.start_vector(g.n, 2), 60)
    a = oracle.cheb_coeffs(0.05 * lmax, lmax, p)
    Rs, R64 = W.signals(g.n, r, seed + 1)
    T = W.unit_rows(g.n, r, seed + 2)
    return g, w64, L, lmax, a, Rs, R64, T


def _oracle_grads(g, w64, L, lmax, a, R64, T, sigma):
    Y = oracle.cheb_filter(L, lmax, a, R64)
    loss, G = oracle.rownorm_loss_grad(Y, T.astype(np.float64))
    dw, da = oracle.cheb_filter_adjoint(g.n, g.row_ptr, g.col_idx, w64, lmax, a, R64, G)
    ds = oracle.dsigma(dw, w64, g.d2.astype(np.float32).astype(np.float64), sigma)
    return Y, loss, G, dw, da, ds


def test_gauss_weights_and_bwd():
    g = W.gmm_knn(3000, 16, 5, 10, 1)
    d2 = to_dev(g.d2)
    w = asc.gauss_weights(d2, 2.0)
    ref = oracle.gauss_weights(g.d2.astype(np.float64), 2.0)
    np.testing.assert_allclose(host(w), ref, rtol=1e-7)
    dW = np.random.default_rng(1).standard_normal(g.nnz).astype(np.float32)
    ds = host(asc.gauss_weights_bwd(d2, w, to_dev(dW), 2.0))[0]
    ds_ref = oracle.dsigma(dW.astype(np.float64), host(w).astype(np.float64), g.d2.astype(np.float64), 2.0)
    assert ds == pytest.approx(ds_ref, rel=1e-12)


def test_rownorm_loss_bwd():
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((5000, 24)).astype(np.float32)
    Y[11] = 0
    T = W.unit_rows(5000, 24, 4)
    loss, G = asc.rownorm_loss_bwd(block_f32(Y), block_f32(T))
    l_ref, G_ref = oracle.rownorm_loss_grad(Y.astype(np.float64), T.astype(np.float64))
    assert host(loss)[0] == pytest.approx(l_ref, rel=1e-12)
    assert rel_fro(host(G), G_ref) <= 1e-6
    assert np.all(host(G)[11] == 0)


@pytest.mark.parametrize("p,c", [(1, 2), (2, 2), (7, 3), (30, 5), (30, 30), (31, 6)])
@pytest.mark.parametrize("r", [5, 16, 40])
def test_filter_bwd_matches_oracle(p, c, r):
    g, w64, L, lmax, a, Rs, R64, T = _problem(n=1500, r=r, p=p)
    G64 = W.signals_f64(g.n, r, 99).astype(np.float32).astype(np.float64)  # G as the GPU receives it
    Gd = upload_graph(g, w=w64.astype(np.float32))
    Rd = block_f32(Rs)
    Y, ck = asc.cheb_filter(Gd, scalar(lmax), to_dev(a), Rd, ckpt_stride=c)
    dW, dc = asc.cheb_filter_bwd(Gd, scalar(lmax), to_dev(a), Rd, ck, c, block_f32(G64))
    # the float32 weights differ from w64 by rounding: compare the adjoint of
    # the operator the GPU applies (oracle on the float32-rounded weights)
    w32 = w64.astype(np.float32).astype(np.float64)
    dw_ref, da_ref = oracle.cheb_filter_adjoint(g.n, g.row_ptr, g.col_idx, w32, lmax, a, R64, G64)
    assert rel_fro(host(dW), dw_ref) <= TOL_DW
    assert rel_fro(host(dc), da_ref) <= TOL_DA


def test_filter_bwd_order_zero_and_no_dw():
    g, w64, L, lmax, a, Rs, R64, T = _problem(n=500, r=8, p=0)
    Gd = upload_graph(g, w=w64.astype(np.float32))
    G64 = W.signals_f64(g.n, 8, 7).astype(np.float32).astype(np.float64)
    Y, ck = asc.cheb_filter(Gd, scalar(lmax), to_dev(a), block_f32(Rs), ckpt_stride=2)
    dW, dc = asc.cheb_filter_bwd(Gd, scalar(lmax), to_dev(a), block_f32(Rs), ck, 2, block_f32(G64))
    assert np.all(host(dW) == 0)
    assert host(dc)[0] == pytest.approx(float(np.sum(G64 * R64)), rel=1e-10)


def test_end_to_end_autograd_matches_oracle():
    sigma = 2.0
    g, w64, L, lmax, a, Rs, R64, T = _problem(n=2500, r=16, p=40, sigma=sigma)
    w32 = oracle.gauss_weights(g.d2.astype(np.float64), sigma).astype(np.float32).astype(np.float64)
    L32 = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, w32)
    Y, loss_ref, G, dw_ref, da_ref, ds_ref = _oracle_grads(g, w32, L32, lmax, a, R64, T, sigma)
    d2 = to_dev(g.d2)
    sig = torch.tensor(sigma, dtype=torch.float64, device=DEV, requires_grad=True)
    coeffs = torch.tensor(a, dtype=torch.float64, device=DEV, requires_grad=True)
    w = GaussWeights.apply(d2, sig)
    w.retain_grad()
    rp = to_dev(g.row_ptr)
    ci = to_dev(g.col_idx)
    Yd = ChebFilter.apply(w, coeffs, rp, ci, scalar(lmax), block_f32(Rs), 7)
    loss = RowNormLoss.apply(Yd, block_f32(T))
    loss.backward()
    assert float(loss.detach().cpu()) == pytest.approx(loss_ref, rel=1e-5)
    assert rel_fro(host(w.grad), dw_ref) <= TOL_DW
    assert rel_fro(host(coeffs.grad), da_ref) <= TOL_DA
    assert float(sig.grad.cpu()) == pytest.approx(ds_ref, rel=TOL_DSIGMA)


def test_bwd_deterministic_and_bf16_runs():
    g, w64, L, lmax, a, Rs, R64, T = _problem(n=1200, r=16, p=20)
    Gd = upload_graph(g, w=w64.astype(np.float32))
    G64 = W.signals_f64(g.n, 16, 3).astype(np.float32).astype(np.float64)
    out = []
    for _ in range(2):
        Y, ck = asc.cheb_filter(Gd, scalar(lmax), to_dev(a), block_f32(Rs), ckpt_stride=4)
        out.append([host(t) for t in asc.cheb_filter_bwd(Gd, scalar(lmax), to_dev(a), block_f32(Rs), ck, 4,
                                                         block_f32(G64))])
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    # bfloat16 states: same interface, looser accuracy (states rounded to 8 bits)
    Rb, Rb64 = W.signals(g.n, 16, 5, "bf16")
    Y, ck = asc.cheb_filter(Gd, scalar(lmax), to_dev(a), block_bf16(Rb), ckpt_stride=4)
    dW, dc = asc.cheb_filter_bwd(Gd, scalar(lmax), to_dev(a), block_bf16(Rb), ck, 4, block_f32(G64))
    w32 = w64.astype(np.float32).astype(np.float64)
    dw_ref, da_ref = oracle.cheb_filter_adjoint(g.n, g.row_ptr, g.col_idx, w32, lmax, a, Rb64, G64)
    print("bf16 bwd rel dW", rel_fro(host(dW), dw_ref), "rel da", rel_fro(host(dc), da_ref))
    assert rel_fro(host(dW), dw_ref) <= 0.1
    assert rel_fro(host(dc), da_ref) <= 0.1


@pytest.mark.parametrize("r,p", [(16, 30), (40, 7), (5, 1)])
def test_state_store_forward_and_backward_equal_checkpoint_path(r, p):
    g, w64, L, lmax, a, Rs, R64, T = _problem(n=1500, r=r, p=p)
    Gd = upload_graph(g, w=w64.astype(np.float32))
    G64 = W.signals_f64(g.n, r, 5).astype(np.float32).astype(np.float64)
    Rd = block_f32(Rs)
    Y1, ck1 = asc.cheb_filter(Gd, scalar(lmax), to_dev(a), Rd, ckpt_stride=1)
    Y3, ck3 = asc.cheb_filter(Gd, scalar(lmax), to_dev(a), Rd, ckpt_stride=3)
    np.testing.assert_array_equal(host(Y1), host(Y3))
    d1 = [host(t) for t in asc.cheb_filter_bwd(Gd, scalar(lmax), to_dev(a), Rd, ck1, 1, block_f32(G64))]
    d3 = [host(t) for t in asc.cheb_filter_bwd(Gd, scalar(lmax), to_dev(a), Rd, ck3, 3, block_f32(G64))]
    np.testing.assert_array_equal(d1[0], d3[0])
    np.testing.assert_array_equal(d1[1], d3[1])
    w32 = w64.astype(np.float32).astype(np.float64)
    dw_ref, da_ref = oracle.cheb_filter_adjoint(g.n, g.row_ptr, g.col_idx, w32, lmax, a, R64, G64)
    assert rel_fro(d1[0], dw_ref) <= TOL_DW
    assert rel_fro(d1[1], da_ref) <= TOL_DA


def test_state_store_layout_is_independent_of_tuning():
    # r = 72: the default 32-column slices give 96 stored columns, 64-column
    # slices would need 128; a store sized before a re-tune must stay valid
    r, p = 72, 12
    g, w64, L, lmax, a, Rs, R64, T = _problem(n=1500, r=r, p=p)
    Gd = upload_graph(g, w=w64.astype(np.float32))
    G64 = W.signals_f64(g.n, r, 5).astype(np.float32).astype(np.float64)
    Rd = block_f32(Rs)
    lib = asc._abi.lib()
    nb = lib.asc_ckpt_bytes(Gd.c(), r, asc.ASC_F32, p, 1)
    states = asc.workspace(nb, DEV)
    Y0, _ = asc.cheb_filter(Gd, scalar(lmax), to_dev(a), Rd, ckpt_stride=1, ckpt=states)
    d0 = [host(t) for t in asc.cheb_filter_bwd(Gd, scalar(lmax), to_dev(a), Rd, states, 1, block_f32(G64))]
    Y0 = host(Y0)
    try:
        asc.tune_set(Gd, r, torch.float32, 64, 4)
        assert lib.asc_ckpt_bytes(Gd.c(), r, asc.ASC_F32, p, 1) == nb
        Y1, ck = asc.cheb_filter(Gd, scalar(lmax), to_dev(a), Rd, ckpt_stride=1, ckpt=states)
        assert ck.data_ptr() == states.data_ptr()
        asc.tune_set(Gd, r, torch.float32, 16, 2)  # re-tuned between forward and backward
        d1 = [host(t) for t in asc.cheb_filter_bwd(Gd, scalar(lmax), to_dev(a), Rd, states, 1, block_f32(G64))]
        _, lam, _, _, _ = asc.lambda_k_filter(Gd, scalar(lmax), 5, p, 8, Rd, None, states)
        assert 0.0 < host(lam)[0] <= lmax
    finally:
        asc.tune_set(Gd, r, torch.float32, 0, 0)
    # the variant bits change only the tile schedule: results are bit-identical
    np.testing.assert_array_equal(host(Y1), Y0)
    np.testing.assert_array_equal(d1[0], d0[0])
    np.testing.assert_array_equal(d1[1], d0[1])
    w32 = w64.astype(np.float32).astype(np.float64)
    dw_ref, da_ref = oracle.cheb_filter_adjoint(g.n, g.row_ptr, g.col_idx, w32, lmax, a, R64, G64)
    assert rel_fro(d1[0], dw_ref) <= TOL_DW
    assert rel_fro(d1[1], da_ref) <= TOL_DA


def test_backward_xcd_band_schedule_gives_the_same_gradients():
    # variant bit 2 changes only which workgroup takes which rows: dW (summed
    # per entry by its own row) is bit-identical, dcoeffs (block partials) equal
    # to rounding
    r, p = 16, 20
    g, w64, L, lmax, a, Rs, R64, T = _problem(n=3000, r=r, p=p)
    Gd = upload_graph(g, w=w64.astype(np.float32))
    G64 = W.signals_f64(g.n, r, 5).astype(np.float32).astype(np.float64)
    Rd = block_f32(Rs)
    _, st0 = asc.cheb_filter(Gd, scalar(lmax), to_dev(a), Rd, ckpt_stride=1)
    d0 = [host(t) for t in asc.cheb_filter_bwd(Gd, scalar(lmax), to_dev(a), Rd, st0, 1, block_f32(G64))]
    try:
        asc.tune_set(Gd, r, torch.float32, 16, 4)
        _, st1 = asc.cheb_filter(Gd, scalar(lmax), to_dev(a), Rd, ckpt_stride=1)
        d1 = [host(t) for t in asc.cheb_filter_bwd(Gd, scalar(lmax), to_dev(a), Rd, st1, 1, block_f32(G64))]
    finally:
        asc.tune_set(Gd, r, torch.float32, 0, 0)
    np.testing.assert_array_equal(d1[0], d0[0])
    np.testing.assert_allclose(d1[1], d0[1], rtol=1e-12, atol=1e-12 * np.max(np.abs(d0[1])))


@pytest.mark.parametrize("c", [1, 4])
@pytest.mark.parametrize("r", [5, 40])
def test_backward_with_tiles_too_long_to_stage(c, r):
    # rows 0..319 form a dense block (about 160 entries per row, so each of
    # its 32-row tiles holds more stored entries than the 4096 the adjoint
    # stages in LDS and stores its accumulator entries directly); the other
    # rows are sparse (staged tiles)
    rng = np.random.default_rng(21)
    n, nd = 2400, 320
    iu = np.triu_indices(nd, 1)
    keep = rng.random(iu[0].shape[0]) < 0.5
    dense = np.stack([iu[0][keep], iu[1][keep]], 1)
    sparse = rng.integers(0, n, size=(8 * n, 2))
    sparse = sparse[sparse[:, 0] != sparse[:, 1]]
    e = np.concatenate([dense, np.sort(sparse, axis=1)])
    e = np.unique(e, axis=0)
    g = W.from_edges(n, e, rng.uniform(0.5, 2.0, size=e.shape[0]))
    per_tile = np.diff(g.row_ptr[::32])
    assert per_tile.max() > 4096 and per_tile.min() <= 4096
    w64 = g.w.astype(np.float64)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, w64)
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, w64)
    lmax = oracle.lmax_estimate(L, s, W.start_vector(g.n, 3), 60)
    p = 12
    a = oracle.cheb_coeffs(0.1 * lmax, lmax, p)
    Rs, R64 = W.signals(g.n, r, 22)
    G64 = W.signals_f64(g.n, r, 23).astype(np.float32).astype(np.float64)
    Gd = upload_graph(g)
    Rd = block_f32(Rs)
    Y, ck = asc.cheb_filter(Gd, scalar(lmax), to_dev(a), Rd, ckpt_stride=c)
    dW, dc = asc.cheb_filter_bwd(Gd, scalar(lmax), to_dev(a), Rd, ck, c, block_f32(G64))
    dw_ref, da_ref = oracle.cheb_filter_adjoint(g.n, g.row_ptr, g.col_idx, w64, lmax, a, R64, G64)
    assert rel_fro(host(dW), dw_ref) <= TOL_DW
    assert rel_fro(host(dc), da_ref) <= TOL_DA
