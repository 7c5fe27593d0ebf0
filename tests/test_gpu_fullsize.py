"""GPU parity at the full benchmark sizes, in the launch configuration the
bench times (autotuned tiling), against the FP64 oracle on samples the oracle
can afford, and by properties that hold at any size."""
import os

import numpy as np
import pytest
import torch

import oracle
import oracle.cpu_baseline as cb
import workloads as W
import paper_1509_08863_amd as asc

from gpu_util import DEV, block_f32, block_bf16, scalar, host, rel_fro, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _c_baseline():
    cb.ensure_built()


def _upload(g, w=None):
    rp = to_dev(g.row_ptr)
    ci = to_dev(g.col_idx)
    wt = to_dev(g.weights_or_ones() if w is None else w)
    return asc.graph_prepare(rp, ci, wt)


# columns of the 96-column block sampled at full size: both ends of each of the
# three 32-column float32 slices (and both sides of the 64-column bfloat16 split)
SAMPLE = [0, 31, 32, 63, 64, 95]


@pytest.fixture(scope="module")
def sbm1e6():
    """The 1M-node SBM on the device with the oracle's lambda_max (40 Lanczos
    iterations from the workload's start vector) and the seeded signals."""
    cfg = W.WORKLOADS[3]
    seeds = W.workload_seeds(3)
    g = W.workload_graph(3)
    print(f"[fullsize] 1M-node SBM: n={g.n} nnz={g.nnz}", flush=True)
    G = _upload(g)
    v0 = W.start_vector(g.n, seeds["lanczos"])
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, None)
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, None)
    lmax_o = oracle.lmax_estimate(L, s, v0, 40)
    del L
    Rs, R64 = W.signals(g.n, cfg["r"], seeds["signals"])
    yield dict(cfg=cfg, seeds=seeds, g=g, G=G, v0=v0, lmax=lmax_o, Rs=Rs, R64=R64)
    del G
    torch.cuda.empty_cache()


def test_sbm_1e6_filter_sampled_columns_and_eigcount_properties(sbm1e6):
    d = sbm1e6
    g, G, cfg, seeds, lmax_o = d["g"], d["G"], d["cfg"], d["seeds"], d["lmax"]
    r, p, k, steps = cfg["r"], cfg["p"], cfg["k"], cfg["steps"]
    R64 = d["R64"]
    R = block_f32(d["Rs"])
    # lambda_max estimate: same Lanczos on the device
    lm_gpu = asc.lmax_estimate(G, to_dev(d["v0"]), 40, host=True)[1]
    assert lm_gpu == pytest.approx(lmax_o, rel=1e-8)
    asc.autotune_filter(G, scalar(lmax_o), R, 2)  # the bench's launch configuration
    a = oracle.cheb_coeffs(0.17 * lmax_o, lmax_o, p)
    Yref = cb.cheb_filter(g.n, g.row_ptr, g.col_idx, None, lmax_o, a, R64[:, SAMPLE])
    Y = host(asc.cheb_filter(G, scalar(lmax_o), to_dev(a), R))
    for q, c in enumerate(SAMPLE):
        e = rel_fro(Y[:, c], Yref[:, q])
        print(f"[fullsize] f32 column {c}: rel err {e:.3e}")
        assert e <= 1e-5, (c, e)
    assert rel_fro(Y[:, SAMPLE], Yref) <= 1e-5
    # bfloat16 states: same columns, stated tolerance
    Rb, Rb64 = W.signals(g.n, r, seeds["signals"], "bf16")
    asc.autotune_filter(G, scalar(lmax_o), block_bf16(Rb), 2)
    Yb = host(asc.cheb_filter(G, scalar(lmax_o), to_dev(a), block_bf16(Rb)))
    Ybref = cb.cheb_filter(g.n, g.row_ptr, g.col_idx, None, lmax_o, a, Rb64[:, SAMPLE])
    for q, c in enumerate(SAMPLE):
        e = rel_fro(Yb[:, c], Ybref[:, q])
        print(f"[fullsize] bf16 column {c}: rel err {e:.3e}")
        assert e <= 6e-2, (c, e)
    # eigenvalue count at full size: mu_0 = |R|_F^2 exactly defined, and the
    # dichotomy brackets k - 1/2 between its last lower and upper cut-offs
    mu = host(asc.cheb_moments(G, scalar(lmax_o), p, R))
    assert mu[0] == pytest.approx(float(np.sum(R64 * R64)), rel=1e-12)
    lam, traj = asc.eigcount_dichotomy(to_dev(mu), scalar(lmax_o), k, steps)
    traj = host(traj)
    hi_counts = [c for (m, c) in traj if c >= k - 0.5]
    lo_counts = [c for (m, c) in traj if c < k - 0.5]
    assert hi_counts and lo_counts
    assert host(lam)[0] == min(m for (m, c) in traj if c >= k - 0.5)


def test_sbm_1e6_one_pass_lambda_k_filter_against_oracle(sbm1e6):
    """The one-pass path the bench times (moments from the recurrence that
    fills the state store, dichotomy and coefficients on the device, Y
    combined from the store) at full size.
    (1) R zero outside the sample columns, in the same 96-column launch: the
        float64 moments of the moment pass and the counts at every trial
        cut-off of the one-pass dichotomy against the oracle's moments of the
        sample columns, and Y on those columns against the oracle filter at
        the GPU's own lambda_k;
    (2) the full block: Y on the sample columns and the coefficients against
        the oracle at the GPU's own lambda_k, the estimate against the
        trajectory's own counts."""
    d = sbm1e6
    g, G, cfg, lmax_o = d["g"], d["G"], d["cfg"], d["lmax"]
    r, p, k, steps = cfg["r"], cfg["p"], cfg["k"], cfg["steps"]
    R64 = d["R64"]
    R = block_f32(d["Rs"])
    asc.autotune_filter(G, scalar(lmax_o), R, 2)
    # (1) sample columns only
    Rz = np.zeros_like(d["Rs"])
    Rz[:, SAMPLE] = d["Rs"][:, SAMPLE]
    Rzd = block_f32(Rz)
    Rz64 = Rz.astype(np.float64)[:, SAMPLE]
    mu_o = cb.cheb_moments(g.n, g.row_ptr, g.col_idx, None, lmax_o, p, Rz64)
    mu = host(asc.cheb_moments(G, scalar(lmax_o), p, Rzd))
    dmu = np.max(np.abs(mu - mu_o)) / mu_o[0]
    print(f"[fullsize] sample moments: max |dmu| / mu_0 = {dmu:.3e}")
    assert dmu <= 1e-5
    Yz, lam_z, traj_z, co_z, st = asc.lambda_k_filter(G, scalar(lmax_o), k, p, steps, Rzd)
    lam_z, traj_z, Yz = host(lam_z)[0], host(traj_z), host(Yz)
    del st
    torch.cuda.empty_cache()
    for s_ in range(steps):
        c_o = oracle.eigcount_from_moments(mu_o, traj_z[s_, 0], lmax_o)
        print(f"[fullsize] one-pass count at {traj_z[s_, 0]:.6f}: {traj_z[s_, 1]:.6f} (oracle {c_o:.6f})")
        assert abs(traj_z[s_, 1] - c_o) <= 1e-5 * mu_o[0]
    hits = [m for (m, c) in traj_z if c >= k - 0.5]
    assert lam_z == (min(hits) if hits else lmax_o)
    a_z = oracle.cheb_coeffs(lam_z, lmax_o, p)
    np.testing.assert_allclose(host(co_z), a_z, rtol=0, atol=1e-13)
    Yz_o = cb.cheb_filter(g.n, g.row_ptr, g.col_idx, None, lmax_o, a_z, Rz64)
    assert rel_fro(Yz[:, SAMPLE], Yz_o) <= 1e-5
    assert np.all(np.delete(Yz, SAMPLE, axis=1) == 0.0)
    # (2) the full block, as timed
    Y, lam, traj, co, st = asc.lambda_k_filter(G, scalar(lmax_o), k, p, steps, R)
    lam, traj, Y = host(lam)[0], host(traj), host(Y)
    del st
    torch.cuda.empty_cache()
    hits = [m for (m, c) in traj if c >= k - 0.5]
    assert hits and len(hits) < steps
    assert lam == min(hits)
    a = oracle.cheb_coeffs(lam, lmax_o, p)
    np.testing.assert_allclose(host(co), a, rtol=0, atol=1e-13)
    Yo = cb.cheb_filter(g.n, g.row_ptr, g.col_idx, None, lmax_o, a, R64[:, SAMPLE])
    for q, c in enumerate(SAMPLE):
        e = rel_fro(Y[:, c], Yo[:, q])
        print(f"[fullsize] one-pass column {c}: rel err {e:.3e}")
        assert e <= 1e-5, (c, e)


def test_sbm_1e6_fwd_bwd_sampled_against_oracle(sbm1e6):
    """fwd+bwd as the bench times it (state store, ckpt_stride = 1) and with
    checkpoints every ceil(sqrt(p)) steps, at full size: dW on 3000 sampled
    stored entries and the coefficient gradients against the float64 adjoint,
    with the upstream gradient G (the row-normalised loss's) kept on three
    columns, one in each 32-column slice, and zero elsewhere, so the oracle
    needs only those columns while the GPU runs the full 96-column block."""
    d = sbm1e6
    g, G, cfg, seeds, lmax_o = d["g"], d["G"], d["cfg"], d["seeds"], d["lmax"]
    r, p = cfg["r"], cfg["p"]
    R64 = d["R64"]
    R = block_f32(d["Rs"])
    cols = [0, 40, 95]
    asc.autotune_filter(G, scalar(lmax_o), R, 2)
    a = oracle.cheb_coeffs(0.17 * lmax_o, lmax_o, p)
    ad = to_dev(a)
    Y, st = asc.cheb_filter(G, scalar(lmax_o), ad, R, ckpt_stride=1)
    target = block_f32(W.unit_rows(g.n, r, seeds["target"]))
    _, Gd = asc.rownorm_loss_bwd(Y, target)
    Gh = host(Gd).astype(np.float32)
    Gz = np.zeros_like(Gh)
    Gz[:, cols] = Gh[:, cols]
    Gzd = block_f32(Gz)
    dW1, dc1 = asc.cheb_filter_bwd(G, scalar(lmax_o), ad, R, st, 1, Gzd)
    dW1, dc1 = host(dW1), host(dc1)
    del st
    torch.cuda.empty_cache()
    c = int(np.ceil(np.sqrt(p)))
    _, ck = asc.cheb_filter(G, scalar(lmax_o), ad, R, ckpt_stride=c)
    dWc, dcc = asc.cheb_filter_bwd(G, scalar(lmax_o), ad, R, ck, c, Gzd)
    dWc, dcc = host(dWc), host(dcc)
    del ck
    torch.cuda.empty_cache()
    ent = np.sort(np.random.default_rng(11).choice(g.nnz, 3000, replace=False))
    print("[fullsize] float64 sampled adjoint on 3 columns", flush=True)
    # unit weights (the device graph has w = NULL): the oracle takes them explicitly
    ones = np.ones(g.nnz, dtype=np.float64)
    dw_o, da_o = oracle.cheb_filter_adjoint_sampled(g.n, g.row_ptr, g.col_idx, ones, lmax_o, a, R64[:, cols],
                                                    Gz[:, cols].astype(np.float64), ent)
    for name, dW, dc in (("store", dW1, dc1), (f"ckpt{c}", dWc, dcc)):
        e_w, e_a = rel_fro(dW[ent], dw_o), rel_fro(dc, da_o)
        print(f"[fullsize] fwd+bwd {name}: dW rel err {e_w:.3e}, dcoeffs rel err {e_a:.3e}")
        assert e_w <= 1e-4
        assert e_a <= 1e-5


def test_sbm_1e5_pipeline_full_parity():
    cfg = W.WORKLOADS[2]
    seeds = W.workload_seeds(2)
    g = W.workload_graph(2)
    r, p, k, steps, iters = cfg["r"], cfg["p"], cfg["k"], cfg["steps"], cfg["kmeans_iters"]
    G = _upload(g)
    Rs, R64 = W.signals(g.n, r, seeds["signals"])
    R = block_f32(Rs)
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, None)
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, None)
    v0 = W.start_vector(g.n, seeds["lanczos"])
    lmax_o = oracle.lmax_estimate(L, s, v0, 60)
    # same iteration, different rounding order: the unconverged tail of the
    # largest Ritz value (no re-orthogonalisation) differs at ~1e-9
    assert asc.lmax_estimate(G, to_dev(v0), 60, host=True)[1] == pytest.approx(lmax_o, rel=1e-8)
    asc.autotune_filter(G, scalar(lmax_o), R, 2)
    # lambda_k: oracle moments + dichotomy vs the one-pass GPU path
    est_o, traj_o = oracle.dichotomy_moments(L, lmax_o, k, p, steps, R64)
    Y, lam, traj, co, _ = asc.lambda_k_filter(G, scalar(lmax_o), k, p, steps, R)
    traj = host(traj)
    tie = False
    for st in range(steps):
        if abs(traj_o[st, 1] - (k - 0.5)) <= 1e-3:
            tie = True
            break
        assert traj[st, 0] == traj_o[st, 0]
        assert abs(traj[st, 1] - traj_o[st, 1]) <= 1e-3
    Yo = cb.cheb_filter(g.n, g.row_ptr, g.col_idx, None, lmax_o, oracle.cheb_coeffs(est_o, lmax_o, p), R64)
    if not tie:
        assert host(lam)[0] == est_o
        assert rel_fro(host(Y), Yo) <= 1e-5
    # normalisation and k-means on the oracle's features (identical inputs)
    Fo, _ = oracle.normalize_rows(Yo)
    Yd = block_f32(Yo.astype(np.float32))
    asc.normalize_features(Yd)
    F32 = Yo.astype(np.float32).astype(np.float64)
    Fo32, _ = oracle.normalize_rows(F32)
    np.testing.assert_allclose(host(Yd), Fo32, rtol=1e-6, atol=1e-7)
    F = block_f32(Fo.astype(np.float32))
    F32 = Fo.astype(np.float32)
    # k-means++ seeding from the same 53-bit draws on both sides: same rows
    U = W.seeding_draws(k, seeds["kmeans"])
    rows = host(asc.kmeans_pp(F, k, to_dev(U.astype(np.int64))))
    rows_o = oracle.kmeans_pp_rows(F32, k, U)
    np.testing.assert_array_equal(rows, rows_o)
    C = asc.kmeans_init_rows(F, to_dev(rows))
    C0 = F32[rows_o]
    np.testing.assert_array_equal(host(C), C0)
    # Lloyd in lockstep: at every iteration the oracle assigns against the
    # GPU's current centroids (labels must be identical: both decide on the
    # float64 definition) and averages the GPU's labels (float64 means rounded
    # to float32: at most one rounding apart, the sums being in another order)
    fmax = float(np.max(np.abs(F32)))
    for it in range(iters):
        Ch = host(C).copy()
        lab_d, _ = asc.kmeans_assign(F, C)
        lab_o, _ = oracle.kmeans_assign(F32, Ch)
        np.testing.assert_array_equal(host(lab_d), lab_o)
        asc.kmeans_update(F, lab_d, C)
        C_o, _ = oracle.kmeans_update(F32, lab_o, Ch)
        C_o32 = C_o.astype(np.float32)
        dC = np.abs(host(C).astype(np.float64) - C_o32.astype(np.float64))
        assert np.all(dC <= np.spacing(np.abs(C_o32)).astype(np.float64) + 1e-12 * fmax), it
    lab = host(asc.kmeans_assign(F, C)[0])
    # the oracle's own chain from the same seeds: a label may differ only where
    # the oracle's best two float64 distances (final centroids) are within
    # 1e-5 relative of each other
    lab_o, C_fin = oracle.kmeans_lloyd(F32, C0, iters)
    diff = np.nonzero(lab != lab_o)[0]
    print(f"[fullsize] k-means: {diff.size} labels differ from the oracle's own chain")
    if diff.size:
        Cf = C_fin.astype(np.float64)
        D = np.stack([np.sum((F32[diff].astype(np.float64) - Cf[c]) ** 2, axis=1) for c in range(k)], 1)
        D.sort(axis=1)
        assert np.all(D[:, 1] - D[:, 0] <= 1e-5 * D[:, 1]), diff


def test_knn_2e5_gradients_sampled_entries():
    cfg = W.WORKLOADS[5]
    seeds = W.workload_seeds(5)
    g = W.workload_graph(5)
    r, p, sigma = cfg["r"], cfg["p"], cfg["sigma"]
    d2 = to_dev(g.d2)
    w = asc.gauss_weights(d2, sigma)
    w64 = oracle.gauss_weights(g.d2.astype(np.float64), sigma)
    np.testing.assert_allclose(host(w), w64, rtol=1e-7)
    # both sides apply the operator of the float32-rounded oracle weights
    w32 = w64.astype(np.float32).astype(np.float64)
    G = asc.graph_prepare(to_dev(g.row_ptr), to_dev(g.col_idx), to_dev(w32.astype(np.float32)))
    L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, w32)
    s = oracle.strength(g.n, g.row_ptr, g.col_idx, w32)
    lmax_o = oracle.lmax_estimate(L, s, W.start_vector(g.n, seeds["lanczos"]), 60)
    a = oracle.cheb_coeffs(0.05 * lmax_o, lmax_o, p)
    Rs, R64 = W.signals(g.n, r, seeds["signals"])
    T = W.unit_rows(g.n, r, seeds["target"]).astype(np.float64)
    R = block_f32(Rs)
    asc.autotune_filter(G, scalar(lmax_o), R, 2)
    Yo = cb.cheb_filter(g.n, g.row_ptr, g.col_idx, w32, lmax_o, a, R64)
    loss_o, Go = oracle.rownorm_loss_grad(Yo, T)
    Y, st = asc.cheb_filter(G, scalar(lmax_o), to_dev(a), R, ckpt_stride=1)
    assert rel_fro(host(Y), Yo) <= 1e-5
    loss, Gd = asc.rownorm_loss_bwd(Y, block_f32(T.astype(np.float32)))
    assert host(loss)[0] == pytest.approx(loss_o, rel=1e-5)
    # the adjoint is a sum over signal columns: with G nonzero in 8 of the 64
    # columns the oracle needs only those 8 while the GPU runs the full block
    c8 = 8
    Gz = np.zeros_like(Go)
    Gz[:, :c8] = Go[:, :c8].astype(np.float32)
    ent = np.sort(np.random.default_rng(3).choice(g.nnz, 3000, replace=False))
    dw_o, da_o = oracle.cheb_filter_adjoint_sampled(g.n, g.row_ptr, g.col_idx, w32, lmax_o, a, R64[:, :c8],
                                                    Gz[:, :c8], ent)
    dW, dc = asc.cheb_filter_bwd(G, scalar(lmax_o), to_dev(a), R, st, 1, block_f32(Gz.astype(np.float32)))
    assert rel_fro(host(dW)[ent], dw_o) <= 1e-4
    assert rel_fro(host(dc), da_o) <= 1e-5


def test_batch_64_graphs_full_size_sampled_graphs():
    cfg = W.WORKLOADS[4]
    r, p, steps = cfg["r"], cfg["p"], cfg["trials"]
    gs = W.batch_graphs()
    ks = np.array([g.k for g in gs], dtype=np.int32)
    lm = []
    for q, g in enumerate(gs):
        L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, None)
        s = oracle.strength(g.n, g.row_ptr, g.col_idx, None)
        lm.append(oracle.lmax_estimate(L, s, W.start_vector(g.n, 500 + q), 40))
    big, off = W.concat_graphs(gs)
    G = _upload(big)
    Rs, R64 = W.signals(big.n, r, 4041)
    B = asc.Batch(G, off, ks, r, torch.float32, p, steps)
    Y = block_f32(np.zeros((big.n, r), np.float32))
    lam = torch.empty(len(gs), dtype=torch.float64, device=DEV)
    traj = torch.empty(len(gs), steps, 2, dtype=torch.float64, device=DEV)
    B.run(to_dev(np.array(lm)), block_f32(Rs), Y, lam, traj, use_graph=True)
    lam, traj, Y = host(lam), host(traj), host(Y)
    B.close()
    sizes = np.array([g.n for g in gs])
    checked = 0
    for q in [int(np.argmin(sizes)), int(np.argsort(sizes)[len(gs) // 2]), int(np.argmax(sizes))]:
        g = gs[q]
        L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, None)
        Rq = R64[off[q]:off[q + 1]]
        est, traj_o = oracle.dichotomy_moments(L, lm[q], int(ks[q]), p, steps, Rq)
        tie = False
        for st in range(steps):
            if abs(traj_o[st, 1] - (ks[q] - 0.5)) <= 1e-3:
                tie = True
                break
            assert traj[q, st, 0] == traj_o[st, 0]
            assert abs(traj[q, st, 1] - traj_o[st, 1]) <= 1e-3
        if tie:
            continue
        assert lam[q] == est
        Yo = cb.cheb_filter(g.n, g.row_ptr, g.col_idx, None, lm[q], oracle.cheb_coeffs(est, lm[q], p), Rq)
        assert rel_fro(Y[off[q]:off[q + 1]], Yo) <= 1e-5
        checked += 1
    assert checked >= 2
