"""Benchmark of the hot path on one MI355X.

One step = one pass of the whole path over one synthetic batch:
strengths -> lambda_max (Lanczos) -> lambda_k (Chebyshev moments + eigenvalue-
count dichotomy) -> coefficients -> polynomial filter of the R random signals
-> row normalisation -> k-means (init rows, iterations of assign + update,
final assign).

Default workload: stochastic block model, N = 1,000,000 nodes, 50 communities
with Dirichlet(5) sizes, mean degree 30, p_out/p_in = 0.05, unit weights
stored as float32; R = 96 signals, order p = 150, 12 dichotomy steps, k = 50,
10 k-means iterations.  Inputs are resident in HBM before timing starts.

Prints ONE JSON line.  `value` is the filter's algorithmic HBM throughput
(GB/s): p x B_step / (measured filter time), with
B_step = 4(N+1) + 8 nnz + 4N + 3 N R b_T + 2 N R 4 (row offsets, column
indices and weights, diagonal, T_j / T_{j-1} / T_{j+1}, read+write of Y).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0

# Memory traffic of one launch of the recurrence step with Y accumulation on
# the 1M-node SBM (one 32-column float32 slice, weights stored), from
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs (KiB per dispatch), scaled by
# the same counters on the plain 2 GiB copy kernel (FETCH_SIZE reads 1 GiB for
# 2 GiB read -> x2.0; WRITE_SIZE reads 2 GiB -> x1.0).  Keyed by the launch
# variant; valid only while the kernel source is the one measured (sha1 of the
# step-kernel region of recurrence.hpp), otherwise reported null.
STEP_TRAFFIC = {
    "src_sha1": "fe387ae335732b0e00bdf449e9fa3432ce6662d3",
    "workload": "sbm_n1e6_k50dir_d30_r96_p150",
    "fetch_scale": 2.0, "write_scale": 1.0,
    # (slice_cols, variant) -> (FETCH_SIZE, WRITE_SIZE) in KiB, average over the
    # 2700 step launches of 6 filters (steps that update Y and steps that do not)
    "kib_per_launch": {(32, 4): (2192537.93, 188338.45)},
}


# The same for the adjoint step of the backward (stored states, dW, da and
# A_j out), averaged over its 1332 launches in 3 fwd+bwd passes on the
# 1M-node SBM (tiles' per-entry accumulator stores staged in LDS).
ADJ_TRAFFIC = {
    "src_sha1": "e9b346b877feb08c35c8a255ea151fb6a542363a",
    "workload": "sbm_n1e6_k50dir_d30_r96_p150",
    "fetch_scale": 2.0, "write_scale": 1.0,
    "kib_per_launch": {(32, 4): (2304920.5, 247664.5)},
}

# The recurrence step on the same graph with each generating block's nodes
# contiguous (block order, round-robin tiles): average over the 2700 step
# launches of 6 filters (steps with and without Y).
BLOCK_STEP_TRAFFIC = {
    "src_sha1": "fe387ae335732b0e00bdf449e9fa3432ce6662d3",
    "workload": "sbm_n1e6_k50dir_d30_r96_p150",
    "fetch_scale": 2.0, "write_scale": 1.0,
    "kib_per_launch": {(32, 0): (2143150.71, 188338.45)},
}


def step_kernel_sha1():
    import hashlib
    src = open(os.path.join(ROOT, "paper_1509_08863_amd", "csrc", "recurrence.hpp")).read()
    a = src.index("// The rest of a row's step for one panel")
    b = src.index("// d_i = 4 s_i / lmax - 2")
    return hashlib.sha1(src[a:b].encode()).hexdigest()


def step_traffic_bytes(workload, slice_cols, variant, t=None):
    """Counter bytes per launch of the tuned step kernel, or None."""
    t = STEP_TRAFFIC if t is None else t
    kib = t["kib_per_launch"].get((slice_cols, variant))
    if kib is None or step_kernel_sha1() != t["src_sha1"] or workload != t["workload"]:
        return None
    return 1024 * (kib[0] * t["fetch_scale"] + kib[1] * t["write_scale"])


def b_step(n, nnz, r, bt, weighted=True):
    return 4 * (n + 1) + nnz * (4 + (4 if weighted else 0)) + 4 * n + 3 * n * r * bt + 2 * n * r * 4


def b_adj_step(n, nnz, r, bt, weighted=True):
    """Algorithmic bytes of one adjoint step over all r columns: the matrix
    (row_ptr, col, w, diagonal), A_{j+1} gathered once, A_{j+2}, A_j written,
    T_j, G (float32), and the per-entry accumulator read and written."""
    b_mat = 4 * (n + 1) + nnz * (4 + (4 if weighted else 0)) + 4 * n
    return b_mat + n * r * (4 * bt + 4) + 8 * nnz


def adj_kernel_sha1():
    import hashlib
    src = open(os.path.join(ROOT, "paper_1509_08863_amd", "csrc", "grad.hip")).read()
    a = src.index("// PF: the next neighbour group's indices")
    b = src.index("template <typename TS, int LPR, bool PF>\nhipError_t launch_adj_t")
    return hashlib.sha1(src[a:b].encode()).hexdigest()


def adj_traffic_bytes(workload, slice_cols, variant):
    """Counter bytes per launch of the adjoint step, or None."""
    t = ADJ_TRAFFIC
    kib = t["kib_per_launch"].get((slice_cols, variant))
    if kib is None or adj_kernel_sha1() != t["src_sha1"] or workload != t["workload"]:
        return None
    return 1024 * (kib[0] * t["fetch_scale"] + kib[1] * t["write_scale"])


def _time(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def planted_ari(labels_dev, planted):
    """Adjusted Rand index of the clustering against the generator's planted
    blocks (scikit-learn; a quality figure of the run, not a parity check)."""
    if planted is None:
        return None
    from sklearn.metrics import adjusted_rand_score
    return round(float(adjusted_rand_score(planted, labels_dev.cpu().numpy())), 4)


def _progress(msg):
    """One line per finished phase on stderr (the JSON line stays alone on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def extra_knn(dev, orders=("generated", "rcm"), device_graph=True):
    """Gaussian-mixture 10-NN graph, N = 2e5, R = 64, p = 100: lambda_k + filter
    in one pass, the filter alone, and forward+backward through the autograd
    wrappers (sigma, weights, coefficients) with every state stored and with
    checkpoints every ceil(sqrt(p)) steps; as generated and in a locality (RCM)
    node order.  The graph is built on the device (asc_knn: exact neighbours
    of the float32 coordinates) unless device_graph is False (host k-d tree on
    the float64 coordinates)."""
    import torch
    import paper_1509_08863_amd as asc
    from paper_1509_08863_amd.autograd import ChebFilter, GaussWeights, RowNormLoss
    cfg = W.WORKLOADS[5]
    seeds = W.workload_seeds(5)
    r, p, k, sigma = cfg["r"], cfg["p"], cfg["k"], cfg["sigma"]
    t0 = time.time()
    if device_graph:
        x, _ = W.gmm_points(cfg["n"], 16, 20, seeds["graph"])
        kg = asc.knn_graph(torch.from_numpy(x.astype(np.float32)).to(dev), 10)
        g0 = W.Graph(n=cfg["n"], row_ptr=kg["row_ptr"].cpu().numpy(), col_idx=kg["col_idx"].cpu().numpy(),
                     d2=kg["d2"].cpu().numpy())
        del kg
    else:
        g0 = W.workload_graph(5)
    out = {"workload": cfg["name"], "n": g0.n, "nnz": g0.nnz, "graph_s": round(time.time() - t0, 2),
           "graph": "device kNN build (asc_knn)" if device_graph else "host k-d tree"}
    c_ck = int(np.ceil(np.sqrt(p)))
    for order in orders:
        t0 = time.time()
        g = g0 if order == "generated" else W.locality_order(g0)[0]
        prep_s = time.time() - t0
        d2 = torch.from_numpy(g.d2).to(dev)
        rp = torch.from_numpy(g.row_ptr).to(dev)
        ci = torch.from_numpy(g.col_idx).to(dev)
        w = asc.gauss_weights(d2, sigma)
        G = asc.graph_prepare(rp, ci, w)
        lmax = asc.lmax_estimate(G, torch.from_numpy(W.start_vector(g.n, seeds["lanczos"])).to(dev), 60)
        R = torch.from_numpy(W.signals(g.n, r, seeds["signals"])[0]).to(dev)
        T = torch.from_numpy(W.unit_rows(g.n, r, seeds["target"])).to(dev)
        tuned = asc.autotune_filter(G, lmax, R, 3)
        Y = torch.empty(g.n, r, dtype=torch.float32, device=dev)
        states = asc.workspace(asc._abi.lib().asc_ckpt_bytes(G.c(), r, asc.ASC_F32, p, 1), dev)
        res, health = {}, {}
        res["ms_lambda_k_filter_one_pass"] = _time(lambda: asc.lambda_k_filter(G, lmax, k, p, 12, R, Y, states))
        health["lambda_k_filter"] = asc.read_flags(asc.lambda_k_filter.last_ws, raise_on_error=False)
        _, lam_k, _, a, _ = asc.lambda_k_filter(G, lmax, k, p, 12, R, Y, states)
        res["ms_filter_fwd"] = _time(lambda: asc.cheb_filter(G, lmax, a, R, Y))
        health["filter"] = asc.read_flags(asc.cheb_filter.last_ws, raise_on_error=False)
        sig = torch.tensor(sigma, dtype=torch.float64, device=dev, requires_grad=True)
        co = a.reshape(-1).clone().requires_grad_(True)
        for label, c in (("store", 1), (f"ckpt{c_ck}", c_ck)):
            def fwd_bwd():
                ww = GaussWeights.apply(d2, sig)
                Yf = ChebFilter.apply(ww, co, rp, ci, lmax, R, c)
                loss = RowNormLoss.apply(Yf, T)
                loss.backward()
                return loss

            res[f"ms_fwd_bwd_autograd_{label}"] = _time(fwd_bwd)
            health[f"fwd_bwd_{label}_backward"] = asc.read_flags(asc.cheb_filter_bwd.last_ws, raise_on_error=False)
            res[f"ckpt_bytes_{label}"] = int(asc._abi.lib().asc_ckpt_bytes(G.c(), r, asc.ASC_F32, p, c))
        bs = b_step(g.n, g.nnz, r, 4)
        res["filter_gbs"] = round(p * bs / (res["ms_filter_fwd"] * 1e-3) / 1e9, 1)
        res["tuned"] = {"slice_cols": tuned[0], "variant": tuned[1]}
        res["reorder_host_s"] = round(prep_s, 3)
        res["health"] = health
        out[order] = {k_: (round(v, 3) if isinstance(v, float) else v) for k_, v in res.items()}
        del states
        torch.cuda.empty_cache()
    return out


def extra_batch(dev):
    """64 SBMs, N log-uniform in [2e3, 2e5], k in 5..40, mean degree 10-30,
    R = 48, p = 80, 8 dichotomy steps, one captured launch of the autotuned
    plan."""
    import torch
    import paper_1509_08863_amd as asc
    cfg = W.WORKLOADS[4]
    r, p, steps = cfg["r"], cfg["p"], cfg["trials"]
    t0 = time.time()
    gs = W.batch_graphs()
    ks = np.array([g.k for g in gs], dtype=np.int32)
    lm = []
    for q, g in enumerate(gs):
        Gq = asc.graph_prepare(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col_idx).to(dev), None)
        lm.append(asc.lmax_estimate(Gq, torch.from_numpy(W.start_vector(g.n, 500 + q)).to(dev), 60))
    lmax = torch.cat(lm)
    big, off = W.concat_graphs(gs)
    gen_s = time.time() - t0
    G = asc.graph_prepare(torch.from_numpy(big.row_ptr).to(dev), torch.from_numpy(big.col_idx).to(dev),
                          torch.from_numpy(big.w).to(dev))
    R = torch.from_numpy(W.signals(big.n, r, 4041)[0]).to(dev)
    Y = torch.empty(big.n, r, dtype=torch.float32, device=dev)
    lam = torch.empty(len(gs), dtype=torch.float64, device=dev)
    traj = torch.empty(len(gs), steps, 2, dtype=torch.float64, device=dev)
    B = asc.Batch(G, off, ks, r, torch.float32, p, steps)
    default_plan = B.info()
    t1 = time.time()
    tuned = B.autotune(lmax, R, Y, lam, traj, probe_runs=1)
    tune_s = time.time() - t1
    ms_graph = _time(lambda: B.run(lmax, R, Y, lam, traj, use_graph=True))
    ms_eager = _time(lambda: B.run(lmax, R, Y, lam, traj, use_graph=False))
    ms_steps = max(1, (p + 1) // 2)
    byts = ms_steps * (b_step(big.n, big.nnz, r, 4) - 8 * big.n * r) + p * b_step(big.n, big.nnz, r, 4)
    info = B.info()
    B.close()
    # the batch raises no device flags: its health is the finiteness of every
    # estimate and of the filtered block
    ok = bool(torch.isfinite(lam).all()) and bool(torch.isfinite(Y).all())
    return {"workload": cfg["name"], "graphs": len(gs), "n_total": big.n, "nnz_total": big.nnz,
            "health": 0 if ok else asc._abi.ASC_FLAG_NONFINITE,
            "ms_per_batch_graph": round(ms_graph, 3), "ms_per_batch_eager": round(ms_eager, 3),
            "gbs": round(byts / (ms_graph * 1e-3) / 1e9, 1), "algorithmic_bytes": byts, "plan": info,
            "default_plan": default_plan, "tuner_ms_per_batch": round(tuned["ms"], 3),
            "tune_s": round(tune_s, 1), "gen_s": round(gen_s, 1)}


def copy_bandwidth(dev, nbytes, reps):
    """Plain 16-byte-vector copy of nbytes (read + write counted)."""
    import torch
    import paper_1509_08863_amd as asc
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    ms = _time(lambda: asc.stream_copy(src, dst), reps)
    del src, dst
    return {"copy_bytes_per_launch": 2 * nbytes, "ms": ms, "GBps": 2 * nbytes / ms / 1e6}


def gather_floor_ms(dev, col_idx, n, reps=20):
    """Time of gathering one 128-byte row per stored entry, in the graph's own
    column-index order, from an n x 32 float32 table: the neighbour-gather
    floor of one 32-column recurrence step."""
    import torch
    import paper_1509_08863_amd as asc
    table = torch.zeros(n, 32, dtype=torch.float32, device=dev)
    sink = torch.zeros(1, dtype=torch.float32, device=dev)
    ms = _time(lambda: asc.gather_probe(table, col_idx, sink), reps)
    del table
    return ms


def extra_stability(dev, c=6, reps_timed=3):
    """Stability measure gamma(k) (Eq. stab): planar Gaussian mixture, kNN
    graph (K = round(ln N)), k over a range, eta_k = 2k, J realisations,
    k-means replicates; the whole sweep as one call."""
    import torch
    import paper_1509_08863_amd as asc
    cfg = W.WORKLOADS[c]
    t0 = time.time()
    g, ks, etas, J, (Rs, _), rows = W.stability_workload(c)
    gen_s = time.time() - t0
    G = asc.graph_prepare(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col_idx).to(dev), None)
    lmax = asc.lmax_estimate(G, torch.from_numpy(W.start_vector(g.n, W.workload_seeds(c)["lanczos"])).to(dev), 60)
    ld = (Rs.shape[1] + 3) // 4 * 4
    R = torch.zeros(g.n, ld, dtype=torch.float32, device=dev)
    R[:, :Rs.shape[1]] = torch.from_numpy(Rs).to(dev)
    R = R[:, :Rs.shape[1]]
    rows_d = torch.from_numpy(rows).to(dev)
    eta_max = max(etas)
    args = (G, lmax, ks[0], ks[-1], etas, J, cfg["reps"], cfg["p"], cfg["steps"], cfg["kmeans_iters"], R, eta_max,
            rows_d)
    out = asc.stability(*args)
    ws = asc.stability.last_ws
    ms = _time(lambda: asc.stability(*args, ws=ws), reps_timed)
    out = asc.stability(*args, ws=ws)
    flags = asc.read_flags(ws, raise_on_error=False)
    gam = out["gamma"].cpu().numpy()
    res = {"workload": cfg["name"], "n": g.n, "nnz": g.nnz, "ks": [ks[0], ks[-1]], "J": J, "reps": cfg["reps"],
           "p": cfg["p"], "kmeans_iters": cfg["kmeans_iters"], "ms_per_sweep": round(ms, 3),
           "gamma": [round(float(x), 4) for x in gam], "k_star": int(ks[int(np.argmax(gam))]),
           "k_true": cfg["k_true"], "workspace_gb": round(ws.numel() / 1e9, 2), "gen_s": round(gen_s, 1),
           "health": flags}
    if cfg["n"] <= 10_000:
        # the oracle on one (k, realisation) cell at the middle k, scaled to the sweep
        import oracle
        L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, None)
        s_o = oracle.strength(g.n, g.row_ptr, g.col_idx, None)
        lmax_o = oracle.lmax_estimate(L, s_o, W.start_vector(g.n, W.workload_seeds(c)["lanczos"]), 60)
        q = len(ks) // 2
        pool = Rs[:, :eta_max].astype(np.float64)
        t0 = time.perf_counter()
        oracle.cluster_once(L, lmax_o, ks[q], etas[q], pool, cfg["p"], cfg["steps"], rows[q, 0],
                            cfg["kmeans_iters"])
        cell_s = time.perf_counter() - t0
        res["cpu_oracle"] = {"s_per_cell": round(cell_s, 2), "cells": len(ks) * J,
                             "s_per_sweep_extrapolated": round(cell_s * len(ks) * J, 1),
                             "sample": f"one realisation at k = {ks[q]} (FP64 NumPy/SciPy, one thread), "
                                       f"scaled by the {len(ks) * J} cells"}
    return res


def extra_small(dev):
    """SBM N = 1000, k = 10, mean degree 16, R = 32, p = 50: latency-bound (the
    working set sits in L2), reported as microseconds per filter."""
    import torch
    import paper_1509_08863_amd as asc
    cfg = W.WORKLOADS[1]
    seeds = W.workload_seeds(1)
    g = W.workload_graph(1)
    G = asc.graph_prepare(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col_idx).to(dev),
                          torch.from_numpy(g.weights_or_ones()).to(dev))
    R = torch.from_numpy(W.signals(g.n, cfg["r"], seeds["signals"])[0]).to(dev)
    lmax = asc.lmax_estimate(G, torch.from_numpy(W.start_vector(g.n, seeds["lanczos"])).to(dev), 60)
    p = cfg["p"]
    # cut-off at lambda_k (k = 10) of the dense Laplacian spectrum (numpy eigvalsh
    # of the 1000 x 1000 L = S - W built from the CSR)
    Ld = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    Ld[rows, g.col_idx] = -g.weights_or_ones().astype(np.float64)
    Ld[np.arange(g.n), np.arange(g.n)] = -Ld.sum(axis=1)
    lam_dense = np.linalg.eigvalsh(Ld)
    lam_k = float(lam_dense[cfg["k"] - 1])
    a = asc.cheb_coeffs(torch.tensor([lam_k], dtype=torch.float64, device=dev), lmax, p)
    Y = torch.empty(g.n, cfg["r"], dtype=torch.float32, device=dev)
    ms = _time(lambda: asc.cheb_filter(G, lmax, a, R, Y), 50)
    ms_lk = _time(lambda: asc.lambda_k_filter(G, lmax, cfg["k"], p, 12, R, Y), 20)
    # the same filter captured once in a HIP graph and replayed (no per-launch host overhead)
    ws = asc.cheb_filter.last_ws
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        with torch.cuda.graph(graph, stream=st):
            asc.cheb_filter(G, lmax, a, R, Y, ws)
    torch.cuda.current_stream().wait_stream(st)
    ms_graph = _time(graph.replay, 50)
    nsl = -(-cfg["r"] // asc.tune_get(G, cfg["r"], torch.float32)[0])
    return {"workload": cfg["name"], "n": g.n, "nnz": g.nnz, "lambda_c": lam_k,
            "lambda_c_source": f"lambda_{cfg['k']} of the dense spectrum (eigvalsh)", "us_per_filter": round(ms * 1e3, 1),
            "step_launches_per_filter": p * nsl, "us_per_step_launch": round(ms * 1e3 / (p * nsl), 2),
            "us_lambda_k_plus_filter_one_pass": round(ms_lk * 1e3, 1), "us_per_filter_graph_replay": round(ms_graph * 1e3, 1)}


def extra_mid(dev):
    """SBM N = 1e5, k = 20, mean degree 20, R = 64, p = 100: the working set
    (about 120 MB) fits the 256 MB Infinity Cache; compared with the copy of a
    64 MiB buffer (cache-resident) as well as with the HBM peak."""
    import torch
    import paper_1509_08863_amd as asc
    cfg = W.WORKLOADS[2]
    seeds = W.workload_seeds(2)
    g = W.workload_graph(2)
    G = asc.graph_prepare(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col_idx).to(dev),
                          torch.from_numpy(g.weights_or_ones()).to(dev))
    r, p = cfg["r"], cfg["p"]
    R = torch.from_numpy(W.signals(g.n, r, seeds["signals"])[0]).to(dev)
    lmax = asc.lmax_estimate(G, torch.from_numpy(W.start_vector(g.n, seeds["lanczos"])).to(dev), 60)
    tuned = asc.autotune_filter(G, lmax, R, 3)
    a = asc.cheb_coeffs(lmax * 0.05, lmax, p)
    Y = torch.empty(g.n, r, dtype=torch.float32, device=dev)
    ms = _time(lambda: asc.cheb_filter(G, lmax, a, R, Y), 10)
    gbs = p * b_step(g.n, g.nnz, r, 4) / (ms * 1e-3) / 1e9
    llc = copy_bandwidth(dev, 64 << 20, 50)["GBps"]
    # lambda_k by dichotomy (12 steps): one moment pass, or one filter pass
    # (without Y) per trial cut-off
    k, steps = cfg["k"], cfg["steps"]
    ms_mom = _time(lambda: asc.eigcount_lambda_k(G, lmax, k, p, steps, R), 5)
    ms_lit = _time(lambda: asc.eigcount_lambda_k(G, lmax, k, p, steps, R, literal=True), 2)
    lam_m, traj_m = asc.eigcount_lambda_k(G, lmax, k, p, steps, R)
    lam_l, traj_l = asc.eigcount_lambda_k(G, lmax, k, p, steps, R, literal=True)
    same = bool(torch.equal(traj_m[:, 0], traj_l[:, 0]))
    # the whole pipeline of this configuration: lambda_k and the filter in one
    # pass, row normalisation, k-means++ seeding (k draws), 10 Lloyd iterations
    U = torch.from_numpy(W.seeding_draws(k, seeds["kmeans"]).astype(np.int64)).to(dev)
    states = asc.workspace(asc._abi.lib().asc_ckpt_bytes(G.c(), r, asc.ASC_F32, p, 1), dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def pipeline(marks=None):
        m = marks if marks is not None else [ev() for _ in range(5)]
        m[0].record()
        asc.lambda_k_filter(G, lmax, k, p, steps, R, Y, states)
        m[1].record()
        asc.normalize_features(Y, want_norms=False)
        m[2].record()
        C = asc.kmeans_init_rows(Y, asc.kmeans_pp(Y, k, U))
        m[3].record()
        for _ in range(cfg["kmeans_iters"]):
            lab, _ = asc.kmeans_assign(Y, C, dist=False)
            asc.kmeans_update(Y, lab, C)
        pipeline.labels = asc.kmeans_assign(Y, C, dist=False)[0]
        m[4].record()
        return m

    pipeline()
    torch.cuda.synchronize()
    runs = [pipeline() for _ in range(5)]
    torch.cuda.synchronize()
    parts = ["lambda_k_filter", "normalize", "kmeanspp", "kmeans"]
    pipe = {nm: round(float(np.mean([m[q].elapsed_time(m[q + 1]) for m in runs])), 3) for q, nm in enumerate(parts)}
    pipe["total"] = round(float(np.mean([m[0].elapsed_time(m[4]) for m in runs])), 3)
    pipe["ari_vs_planted"] = planted_ari(pipeline.labels, g.labels)
    # the same pipeline on the normalised Laplacian (lambda_max = 2)
    two = torch.tensor([2.0], dtype=torch.float64, device=dev)
    Gn = asc.graph_normalized(G)

    def pipeline_n():
        asc.lambda_k_filter(Gn, two, k, p, steps, R, Y, states)
        asc.normalize_features(Y, want_norms=False)
        C = asc.kmeans_init_rows(Y, asc.kmeans_pp(Y, k, U))
        for _ in range(cfg["kmeans_iters"]):
            lab, _ = asc.kmeans_assign(Y, C, dist=False)
            asc.kmeans_update(Y, lab, C)
        return asc.kmeans_assign(Y, C, dist=False)[0]

    pipeline_n()
    ms_n = _time(pipeline_n, 5)
    pipe["normalized_laplacian"] = {"ms_total": round(ms_n, 3), "ari_vs_planted": planted_ari(pipeline_n(), g.labels)}
    del states
    return {"workload": cfg["name"], "n": g.n, "nnz": g.nnz, "ms_per_filter_fwd": round(ms, 3),
            "pipeline_ms": pipe,
            "gbs": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
            "copy_gbs_64MiB": round(llc, 1), "frac_of_cache_resident_copy": round(gbs / llc, 4),
            "tuned": {"slice_cols": tuned[0], "variant": tuned[1]},
            "lambda_k": {"k": k, "steps": steps, "ms_moments": round(ms_mom, 3), "ms_literal": round(ms_lit, 3),
                         "estimate_moments": float(lam_m.cpu()[0]), "estimate_literal": float(lam_l.cpu()[0]),
                         "same_trajectory": same}}


def extra_knn_build(dev, n=200_000, d=16, k=10):
    """K-nearest-neighbour graph of the gradient workload's points (16-D,
    20-component mixture), built on the device: float32 MFMA proposals over
    all pairs, float64 selection, union graph; then Gaussian weights."""
    import torch
    import paper_1509_08863_amd as asc
    x, _ = W.gmm_points(n, d, 20, W.workload_seeds(5)["graph"])
    X = torch.from_numpy(x.astype(np.float32)).to(dev)
    out = asc.knn_graph(X, k)
    ms = _time(lambda: asc.knn_graph(X, k), 3)
    t0 = time.time()
    W.gmm_knn(n, d, 20, k, W.workload_seeds(5)["graph"])
    host_s = time.time() - t0
    import oracle
    t0 = time.time()
    oracle.knn_exact(x.astype(np.float32), k)
    oracle_s = time.time() - t0
    flops = 2.0 * n * n * ((d + 3) // 4 * 4)
    return {"n": n, "d": d, "k": k, "nnz": int(out["col_idx"].numel()), "ms_graph": round(ms, 3),
            "fallback_rows": int(out["fallback_rows"].cpu()[0]),
            "mfma_tflops_whole_build": round(flops / (ms * 1e-3) / 1e12, 2), "mfma_fp32_peak_tflops": 157.3,
            "host_kdtree_s": round(host_s, 2), "cpu_oracle_s": round(oracle_s, 2)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=3, choices=[2, 3],
                    help="3: the 1e6-node SBM (R = 96, p = 150); 2: the 1e5-node SBM (R = 64, p = 100)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the FP64 error check")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--cpu-cols", type=int, default=24,
                    help="columns of R (spread evenly over all slices) for the error check and the CPU baseline")
    ap.add_argument("--no-bwd", action="store_true", help="skip the fwd+bwd timing")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-graph batch")
    ap.add_argument("--no-small", action="store_true", help="skip the 1000-node and 1e5-node SBMs")
    ap.add_argument("--no-normalized", action="store_true",
                    help="skip the pipeline step on the normalised Laplacian")
    ap.add_argument("--no-knn", action="store_true", help="skip the kNN-graph gradient workload")
    ap.add_argument("--no-block-order", action="store_true",
                    help="skip the filter on the block-contiguous node order")
    ap.add_argument("--order", default="generated", choices=["generated", "block"],
                    help="node order of the graph (block: each generating block contiguous)")
    ap.add_argument("--no-pattern", action="store_true", help="skip the pattern-only (w = NULL) filter timing")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (default tiling)")
    ap.add_argument("--extra", action="store_true",
                    help="also time the kNN graph build and the gamma(k) sweep on the 1e5-point mixture")
    ap.add_argument("--no-stability", action="store_true", help="skip the gamma(k) sweep on the 5000-point mixture")
    ap.add_argument("--copy-probe", action="store_true", help="only time the plain 2 GiB copy kernel and exit")
    ap.add_argument("--knn-only", action="store_true", help="only time the kNN graph construction and exit")
    ap.add_argument("--batch-only", action="store_true", help="only time the 64-graph batch and exit")
    ap.add_argument("--knn-grad-only", action="store_true", help="only time the kNN-gradient workload and exit")
    ap.add_argument("--stability-only", type=int, default=0, metavar="C",
                    help="only time the stability sweep of configuration C (6 or 7) and exit")
    ap.add_argument("--fwd-bwd-only", action="store_true",
                    help="only time forward (states stored) + loss + backward on the main graph and exit")
    ap.add_argument("--filter-only", action="store_true",
                    help="only run float32 filters of the headline graph (counter runs) and exit")
    ap.add_argument("--tune", default=None, metavar="RS,VAR",
                    help="fixed float32 launch configuration (slice columns, variant) instead of the autotuner")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_1509_08863_amd as asc

    dev = "cuda:0"
    if args.copy_probe:
        print(json.dumps(copy_bandwidth(dev, 2 << 30, 10)))
        return
    if args.knn_only:
        print(json.dumps(extra_knn_build(dev)))
        return
    if args.batch_only:
        print(json.dumps(extra_batch(dev)))
        return
    if args.knn_grad_only:
        print(json.dumps(extra_knn(dev)))
        return
    if args.stability_only:
        print(json.dumps(extra_stability(dev, args.stability_only)))
        return
    cfg = W.WORKLOADS[args.workload]
    seeds = W.workload_seeds(args.workload)
    t0 = time.time()
    g = W.workload_graph(args.workload)
    _progress(f"graph {cfg['name']}: n={g.n} nnz={g.nnz}")
    order_perm = None
    if args.order == "block":
        g, order_perm = W.block_order(g)
        _progress("nodes relabelled block by block")
    n, nnz, r, p, k = g.n, g.nnz, cfg["r"], cfg["p"], cfg["k"]
    steps_dich, km_iters = cfg["steps"], cfg["kmeans_iters"]
    R32, R64 = W.signals(n, r, seeds["signals"])
    Rbf, Rbf64 = W.signals(n, r, seeds["signals"], "bf16")
    v0 = W.start_vector(n, seeds["lanczos"])
    if order_perm is not None:
        R32, R64, Rbf, Rbf64, v0 = (x[order_perm] for x in (R32, R64, Rbf, Rbf64, v0))
    init = W.init_rows(n, k, seeds["kmeans"])
    gen_s = time.time() - t0

    rp = torch.from_numpy(g.row_ptr).to(dev)
    ci = torch.from_numpy(g.col_idx).to(dev)
    w = torch.from_numpy(g.weights_or_ones()).to(dev)
    G = asc.graph_prepare(rp, ci, w)
    R = torch.from_numpy(R32).to(dev)
    Rb = torch.from_numpy(Rbf.view(np.int16)).to(dev).view(torch.bfloat16)
    v0d = torch.from_numpy(v0).to(dev)
    initd = torch.from_numpy(init).to(dev)
    Y = torch.empty(n, r, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    tuned = {}
    if args.tune:
        rs_, var_ = (int(x) for x in args.tune.split(","))
        asc.tune_set(G, r, torch.float32, rs_, var_)
        tuned["f32"] = (rs_, var_, float("nan"))
    elif not args.no_tune:
        lm0 = asc.lmax_estimate(G, v0d, 60)
        tuned["f32"] = asc.autotune_filter(G, lm0, R, 2)
    if not args.no_tune and not args.no_bf16:
        lm0 = asc.lmax_estimate(G, v0d, 60)
        tuned["bf16"] = asc.autotune_filter(G, lm0, Rb, 2)

    if args.filter_only:
        # the filter alone at lambda_c = 0.17 lambda_max (2 untimed + 3 timed)
        lm = asc.lmax_estimate(G, v0d, 60)
        a = asc.cheb_coeffs(lm * 0.17, lm, p)
        for _ in range(2):
            asc.cheb_filter(G, lm, a, R, Y)
        ms = _time(lambda: asc.cheb_filter(G, lm, a, R, Y), 3)
        print(json.dumps({"workload": cfg["name"], "node_order": args.order, "ms_per_filter_fwd": round(ms, 4),
                          "tuned": tuned.get("f32")}))
        return
    if args.fwd_bwd_only:
        # forward with every state stored, loss, backward (1 untimed + 2 timed)
        lm = asc.lmax_estimate(G, v0d, 60)
        a = asc.cheb_coeffs(lm * 0.17, lm, p)
        st = asc.workspace(asc._abi.lib().asc_ckpt_bytes(G.c(), r, asc.ASC_F32, p, 1), dev)
        target = torch.from_numpy(W.unit_rows(n, r, seeds["target"])).to(dev)

        def fb1():
            Yf, _ = asc.cheb_filter(G, lm, a, R, Y, ckpt_stride=1, ckpt=st)
            _, Gr_ = asc.rownorm_loss_bwd(Yf, target)
            asc.cheb_filter_bwd(G, lm, a, R, st, 1, Gr_)

        ms = _time(fb1, 2)
        print(json.dumps({"workload": cfg["name"], "node_order": args.order, "ms_fwd_bwd_store": round(ms, 4),
                          "tuned": tuned.get("f32")}))
        return

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    L_ = asc._abi.lib()
    health = {}

    def flags_of(name, ws):
        # device health flags of the last run that used ws (synchronises)
        health[name] = asc.read_flags(ws, raise_on_error=False)

    comp_names = ["prepare", "lmax", "lambda_k_coeffs_filter", "-", "-", "normalize", "kmeans"]
    states = asc.workspace(asc._abi.lib().asc_ckpt_bytes(G.c(), r, asc.ASC_F32, p, 1), dev)

    def step(rec=None):
        marks = [ev() for _ in range(len(comp_names) + 1)]
        marks[0].record()
        Gs = asc.graph_prepare(rp, ci, w)
        marks[1].record()
        lmax = asc.lmax_estimate(Gs, v0d, 60)
        marks[2].record()
        # lambda_k (moments + dichotomy), coefficients and the filter in one
        # recurrence pass over a store of all states
        _, lam_k, _, a, _ = asc.lambda_k_filter(Gs, lmax, k, p, steps_dich, R, Y, states)
        marks[3].record()
        marks[4].record()
        marks[5].record()
        asc.normalize_features(Y, want_norms=False)
        marks[6].record()
        C = asc.kmeans_init_rows(Y, initd)
        for _ in range(km_iters):
            lab, _ = asc.kmeans_assign(Y, C, dist=False)
            asc.kmeans_update(Y, lab, C)
        lab, _ = asc.kmeans_assign(Y, C, dist=False)
        marks[7].record()
        if rec is not None:
            rec.append(marks)
        return lmax, lam_k, lab

    _progress(f"tuned {tuned}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    recs = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        out = step(recs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    flags_of("pipeline_lambda_k_filter", asc.lambda_k_filter.last_ws)
    comp = {nm: 0.0 for nm in comp_names if nm != "-"}
    for marks in recs:
        for q, nm in enumerate(comp_names):
            if nm != "-":
                comp[nm] += marks[q].elapsed_time(marks[q + 1]) / len(recs)
    ms_step = wall * 1e3 / args.steps
    lmax_h = float(out[0].cpu()[0])
    lam_k_h = float(out[1].cpu()[0])
    ari_planted = planted_ari(out[2], g.labels)

    # filter alone (fp32 and bf16), events on the launch stream
    # 3 warm-up filters, then 20 back-to-back filters with an event between
    # each: mean (the reported rate), median and min per filter
    def time_filter(Rin, name, reps=20, warm=3):
        a = asc.cheb_coeffs(out[1], out[0], p)
        fws = asc.workspace(L_.asc_filter_workspace(n, r, asc._dtype_code(Rin), p), dev)
        for _ in range(warm):
            asc.cheb_filter(G, out[0], a, Rin, Y, fws)
        torch.cuda.synchronize()
        es = [ev() for _ in range(reps + 1)]
        es[0].record()
        for q in range(reps):
            asc.cheb_filter(G, out[0], a, Rin, Y, fws)
            es[q + 1].record()
        torch.cuda.synchronize()
        flags_of(name, fws)
        each = [es[q].elapsed_time(es[q + 1]) for q in range(reps)]
        return float(np.mean(each)), {"median": round(float(np.median(each)), 4), "min": round(min(each), 4),
                                      "reps": reps}

    _progress(f"{args.steps} pipeline steps: {ms_step:.1f} ms/step")

    # the same step on the normalised Laplacian I - S^-1/2 W S^-1/2 (the
    # variant of the footnote of Sec. 2.1; lambda_max = 2 is known, so no
    # Lanczos), k-means seeded by k-means++: the clustering quality against the
    # planted blocks, which the combinatorial L of these sparse graphs does not
    # reach (its lowest eigenvectors sit on low-degree nodes)
    norm_res = None
    if not args.no_normalized:
        two = torch.tensor([2.0], dtype=torch.float64, device=dev)
        Ukpp = torch.from_numpy(W.seeding_draws(k, seeds["kmeans"]).astype(np.int64)).to(dev)

        def step_norm():
            Gs = asc.graph_prepare(rp, ci, w)
            Gn = asc.graph_normalized(Gs)
            _, lam_n, _, _, _ = asc.lambda_k_filter(Gn, two, k, p, steps_dich, R, Y, states)
            asc.normalize_features(Y, want_norms=False)
            C = asc.kmeans_init_rows(Y, asc.kmeans_pp(Y, k, Ukpp))
            for _ in range(km_iters):
                lab_n, _ = asc.kmeans_assign(Y, C, dist=False)
                asc.kmeans_update(Y, lab_n, C)
            lab_n, _ = asc.kmeans_assign(Y, C, dist=False)
            return lam_n, lab_n

        step_norm()
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(2):
            lam_n, lab_n = step_norm()
        e1.record()
        torch.cuda.synchronize()
        flags_of("pipeline_normalized_lambda_k_filter", asc.lambda_k_filter.last_ws)
        norm_res = {"ms_per_step": round(e0.elapsed_time(e1) / 2, 3), "lambda_max": 2.0,
                    "lambda_k_est": float(lam_n.cpu()[0]), "ari_vs_planted": planted_ari(lab_n, g.labels),
                    "kmeans_seeding": "k-means++ (device draw)"}
        _progress(f"normalised-Laplacian step {norm_res['ms_per_step']:.1f} ms, ARI {norm_res['ari_vs_planted']}")
    ms_f32, stats_f32 = time_filter(R, "filter_f32")
    ms_bf16, stats_bf16 = (None, None) if args.no_bf16 else time_filter(Rb, "filter_bf16")
    # pattern-only graph (w = NULL: unit weights, no weight stream), same plan
    # k-means++ seeding of the same features (k draws), for callers that want
    # it instead of the uniform initial rows the pipeline step uses
    Ud = torch.from_numpy(W.seeding_draws(k, seeds["kmeans"]).astype(np.int64)).to(dev)
    ms_kpp = _time(lambda: asc.kmeans_pp(Y, k, Ud), 3)
    ms_pat = None
    if not args.no_pattern:
        G_pat = asc.graph_prepare(rp, ci, None)
        a_pat = asc.cheb_coeffs(out[1], out[0], p)
        pws = asc.workspace(L_.asc_filter_workspace(n, r, asc.ASC_F32, p), dev)
        ms_pat = _time(lambda: asc.cheb_filter(G_pat, out[0], a_pat, R, Y, pws), 3)
        flags_of("filter_pattern_only", pws)
        del G_pat, pws

    # forward + backward: filter keeping its states, row-normalised loss
    # against a fixed unit-row target, adjoint (edge-weight and coefficient
    # gradients); once with every state stored (ckpt_stride = 1: nothing is
    # recomputed) and once with checkpoint pairs every ceil(sqrt(p)) steps
    # (each segment recomputed once in the backward)
    fb = None
    if not args.no_bwd:
        target = torch.from_numpy(W.unit_rows(n, r, seeds["target"])).to(dev)
        a = asc.cheb_coeffs(out[1], out[0], p)
        fws = asc.workspace(L_.asc_filter_workspace(n, r, asc.ASC_F32, p), dev)
        c_ck = int(np.ceil(np.sqrt(p)))
        fb = {}
        for label, c in (("store", 1), (f"ckpt{c_ck}", c_ck)):
            ck_bytes = int(L_.asc_ckpt_bytes(G.c(), r, asc.ASC_F32, p, c))
            ck = states if c == 1 else asc.workspace(ck_bytes, dev)
            bws = asc.workspace(L_.asc_filter_bwd_workspace(n, nnz, r, asc.ASC_F32, p, c), dev)

            def run_fb():
                Yf, _ = asc.cheb_filter(G, out[0], a, R, Y, fws, ckpt_stride=c, ckpt=ck)
                _, Gr_ = asc.rownorm_loss_bwd(Yf, target)
                asc.cheb_filter_bwd(G, out[0], a, R, ck, c, Gr_, ws=bws)
                return Gr_

            Gr = run_fb()
            torch.cuda.synchronize()
            reps = 2
            e0, e1, b0, b1 = ev(), ev(), ev(), ev()
            e0.record()
            for _ in range(reps):
                Gr = run_fb()
            e1.record()
            # the backward alone (with checkpoints: segment recomputation included)
            b0.record()
            for _ in range(reps):
                asc.cheb_filter_bwd(G, out[0], a, R, ck, c, Gr, ws=bws)
            b1.record()
            torch.cuda.synchronize()
            flags_of(f"fwd_bwd_{label}_forward", fws)
            flags_of(f"fwd_bwd_{label}_backward", bws)
            fb[label] = {"ckpt_stride": c, "ms": round(e0.elapsed_time(e1) / reps, 3),
                         "ms_backward": round(b0.elapsed_time(b1) / reps, 3), "ckpt_bytes": ck_bytes,
                         "backward_ws_bytes": int(bws.numel())}
            del bws, ck
            torch.cuda.empty_cache()
        _progress(f"filter {ms_f32:.1f} ms, fwd+bwd {fb['store']['ms']:.1f} ms (store), "
                  f"{fb[f'ckpt{c_ck}']['ms']:.1f} ms (ckpt {c_ck})")
        del fws
    ms_fb = None if fb is None else fb["store"]["ms"]
    bs32 = b_step(n, nnz, r, 4)
    bs16 = b_step(n, nnz, r, 2)
    bs_pat = b_step(n, nnz, r, 4, weighted=False)
    gbs32 = p * bs32 / (ms_f32 * 1e-3) / 1e9
    gbs16 = None if ms_bf16 is None else p * bs16 / (ms_bf16 * 1e-3) / 1e9

    # error against FP64 on a column sample, same launch configuration
    err = {}
    cpu = None
    if not args.no_check or not args.no_cpu_baseline:
        import oracle
        import oracle.cpu_baseline as cb
        if not os.path.exists(cb.LIB):
            cb.build()
        L = oracle.laplacian_sparse(n, g.row_ptr, g.col_idx, None)
        s = oracle.strength(n, g.row_ptr, g.col_idx, None)
        lmax_o = oracle.lmax_estimate(L, s, v0, 60)
        lc_o = 0.17 * lmax_o
        a_o = oracle.cheb_coeffs(lc_o, lmax_o, p)
        # columns spread evenly over the block, so every slice of every launch plan is sampled
        cidx = np.unique(np.linspace(0, r - 1, min(args.cpu_cols, r)).round().astype(np.int64))
        cols = len(cidx)
        t1 = time.perf_counter()
        Yref = cb.cheb_filter(n, g.row_ptr, g.col_idx, None, lmax_o, a_o, R64[:, cidx])
        cpu_s = time.perf_counter() - t1
        ad = torch.from_numpy(a_o).to(dev)
        ld = torch.tensor([lmax_o], dtype=torch.float64, device=dev)
        Yg = asc.cheb_filter(G, ld, ad, R, Y)[:, cidx].cpu().numpy().astype(np.float64)
        err["f32"] = float(np.linalg.norm(Yg - Yref) / np.linalg.norm(Yref))
        if ms_bf16 is not None:
            Ybref = cb.cheb_filter(n, g.row_ptr, g.col_idx, None, lmax_o, a_o, Rbf64[:, cidx])
            Ygb = asc.cheb_filter(G, ld, ad, Rb, Y)[:, cidx].cpu().numpy().astype(np.float64)
            err["bf16_vs_fp64_on_bf16_R"] = float(np.linalg.norm(Ygb - Ybref) / np.linalg.norm(Ybref))
            err["bf16_vs_fp64_on_fp64_R"] = float(np.linalg.norm(Ygb - Yref) / np.linalg.norm(Yref))
        err["lambda_max_rel"] = abs(lmax_h - lmax_o) / lmax_o  # same start vector, 60 iterations each
        err["sample"] = (f"{cols} columns of R spread over all slices ({cidx[0]}, {cidx[1]}, ..., {cidx[-1]}), "
                         f"lambda_max = oracle Lanczos (60 it), lambda_c = 0.17 lambda_max")
        if not args.no_cpu_baseline:
            ms_cpu_full = cpu_s * 1e3 * (r / cols)  # the recurrence is independent per column
            threads = cb.num_threads()
            cpu = {"value": p * bs32 / (ms_cpu_full * 1e-3) / 1e9, "unit": "GB/s", "cores": threads,
                   "kind": "oracle", "ms_per_filter_extrapolated": ms_cpu_full, "cpu_model": cb.cpu_model(),
                   "sample": f"FP64 C/OpenMP recurrence on {cols} of {r} columns (spread), full graph, p={p}, "
                             f"{cpu_s:.1f} s; scaled by {r}/{cols} to one filter"}
            # the same oracle on one thread, one column
            cb.set_threads(1)
            t1 = time.perf_counter()
            cb.cheb_filter(n, g.row_ptr, g.col_idx, None, lmax_o, a_o, R64[:, :1])
            s1 = time.perf_counter() - t1
            cb.set_threads(threads)
            ms1 = s1 * 1e3 * r
            cpu["single_thread"] = {"value": p * bs32 / (ms1 * 1e-3) / 1e9, "ms_per_filter_extrapolated": ms1,
                                    "sample": f"1 of {r} columns on 1 thread, {s1:.1f} s; scaled by {r}"}

    # per-launch roofline of the step kernel: one launch = one recurrence step
    # over one slice of rs columns; the algorithmic bytes of a step are shared
    # out over its slices (the CSR stream counts once per step).  The filter's
    # other kernels (diagonal, panel packing) take < 0.2% of its time.
    rs32, var32 = tuned.get("f32", (32, 0))[:2]
    nsl = -(-r // rs32)
    launches = p * nsl
    launch_ms = ms_f32 / launches
    alg_launch = bs32 / nsl
    traffic = step_traffic_bytes(cfg["name"], rs32, var32)
    copy_big = copy_bandwidth(dev, 4 << 30, 10)
    copy_llc = copy_bandwidth(dev, 64 << 20, 50)
    gfloor = gather_floor_ms(dev, ci, n) if rs32 == 32 else None
    # Y moves on every other step with float32 states (a pair of terms added
    # at once): the bytes the kernel must move, besides the method's own count
    alg_launch_ymoved = (bs32 - 4 * n * r) / nsl

    # adjoint step of the backward (stored states: p launches per slice)
    fb_roof = None
    if fb is not None:
        # with stored states the backward runs on the store's slice width: the
        # least float32 width (8, 16, 32) covering r, at most 32 columns
        rs_b = 8
        while rs_b < r and rs_b < 32:
            rs_b *= 2
        nsl_b = -(-r // rs_b)
        adj_launch_ms = fb["store"]["ms_backward"] / (p * nsl_b)
        b_adj = b_adj_step(n, nnz, r, 4)
        adj_alg = b_adj / nsl_b
        adj_traffic = adj_traffic_bytes(cfg["name"], rs_b, var32)
        fb_bytes = p * bs32 + 12 * n * r + p * b_adj  # forward, loss, adjoint
        fb_roof = {"bound": "hbm", "kernel": "adj_step", "achieved": round(adj_alg / (adj_launch_ms * 1e-3) / 1e9, 2),
                   "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": round(adj_alg / (adj_launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "traffic": None if adj_traffic is None else round(adj_traffic),
                   "traffic_kind": "L2-to-fabric bytes per launch (FETCH_SIZE x2 + WRITE_SIZE x1), "
                                   "Infinity Cache hits included",
                   "algorithmic_bytes_per_launch": round(adj_alg), "launch_ms": round(adj_launch_ms, 5),
                   "launches_per_backward": p * nsl_b,
                   "whole_fwd_bwd_algorithmic_bytes": fb_bytes,
                   "whole_fwd_bwd_gbs": round(fb_bytes / (fb["store"]["ms"] * 1e-3) / 1e9, 1),
                   "whole_fwd_bwd_frac": round(fb_bytes / (fb["store"]["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        fb["roofline"] = fb_roof

    # the other workloads, compact: the 64-graph batch and the kNN-graph
    # gradient workload (filter, one-pass lambda_k, fwd+bwd stored / checkpointed)
    small_res = mid_res = None
    if not args.no_small:
        small_res = extra_small(dev)
        mid_res = extra_mid(dev)
        _progress(f"1000-node SBM {small_res['us_per_filter']:.0f} us, 1e5-node SBM {mid_res['ms_per_filter_fwd']:.2f} ms")
    if not args.no_batch:
        batch_res = extra_batch(dev)
        health["batch"] = batch_res.pop("health")
        _progress(f"batch {batch_res['ms_per_batch_graph']:.1f} ms")
    else:
        batch_res = None
    if not args.no_knn:
        knn_res = extra_knn(dev, orders=("generated", "rcm"), device_graph=True)
        for o in ("generated", "rcm"):
            for k_, v in knn_res[o].pop("health").items():
                health[f"knn_{o}_{k_}"] = v
        _progress("kNN gradients done")
    else:
        knn_res = None
    # the stability measure gamma(k) over k = 2..20 (Sec. 4.3, the paper's
    # Fig. 2 setting on the planar-mixture stand-in)
    stab_res = None
    if not args.no_stability:
        stab_res = extra_stability(dev, 6)
        health["stability"] = stab_res.pop("health")
        _progress(f"stability sweep {stab_res['ms_per_sweep']:.1f} ms")
    # the same graph with every generating block contiguous (the generator's
    # labels: the best node order a partitioner could find), the filter alone;
    # run last because its tuning entry replaces this graph size's entry
    blk = None
    if not args.no_block_order and args.order == "generated" and g.labels is not None:
        t0 = time.time()
        gb, permb = W.block_order(g)
        reorder_s = time.time() - t0
        Gb = asc.graph_prepare(torch.from_numpy(gb.row_ptr).to(dev), torch.from_numpy(gb.col_idx).to(dev),
                               torch.from_numpy(gb.weights_or_ones()).to(dev))
        Rk = torch.from_numpy(R32[permb]).to(dev)
        tb = asc.autotune_filter(Gb, out[0], Rk, 2)
        ab = asc.cheb_coeffs(out[1], out[0], p)
        bws = asc.workspace(L_.asc_filter_workspace(n, r, asc.ASC_F32, p), dev)
        ms_b = _time(lambda: asc.cheb_filter(Gb, out[0], ab, Rk, Y, bws), 5)
        flags_of("filter_block_order", bws)
        nsl_k = -(-r // tb[0])
        tr_b = step_traffic_bytes(cfg["name"], tb[0], tb[1], BLOCK_STEP_TRAFFIC)
        blk = {"ms_per_filter_fwd": round(ms_b, 4), "gbs": round(p * bs32 / (ms_b * 1e-3) / 1e9, 2),
               "frac": round(p * bs32 / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "launch_ms": round(ms_b / (p * nsl_k), 5), "tuned": {"slice_cols": tb[0], "variant": tb[1]},
               "traffic": None if tr_b is None else round(tr_b),
               "amplification": None if tr_b is None else round(tr_b / (bs32 / nsl_k), 3),
               "reorder_host_s": round(reorder_s, 2),
               "order": "nodes of each generating block contiguous (the generator's labels)"}
        del Gb, Rk, bws
        _progress(f"block order filter {ms_b:.1f} ms")
    extra = None
    if args.extra:
        parts = [("knn_build", lambda: extra_knn_build(dev)), ("stability_large", lambda: extra_stability(dev, 7, 1))]
        extra = {}
        for name, fn in parts:
            extra[name] = fn()
            _progress(f"extra {name} done")
    line = {
        "metric": "Chebyshev-filter SpMM HBM GB/s + ms/filter (fwd, fwd+bwd) at err vs FP64",
        "value": round(gbs32, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "node_order": args.order, "seeds": seeds, "n": n, "nnz": nnz, "r": r,
                   "p": p, "k": k,
                   "dichotomy_steps": steps_dich, "kmeans_iters": km_iters},
        "ms_per_filter_fwd": round(ms_f32, 4),
        "ms_per_filter_fwd_stats": stats_f32,
        "ms_per_filter_fwd_bwd": None if ms_fb is None else round(ms_fb, 4),
        "fwd_bwd": fb,
        "tuned": {k_: {"slice_cols": v[0], "variant": v[1], "ms_per_step": round(v[2], 4)} for k_, v in tuned.items()},
        "err_vs_fp64": err,
        "bf16": None if ms_bf16 is None else {"ms_per_filter_fwd": round(ms_bf16, 4), "gbs": round(gbs16, 2),
                                              "ms_per_filter_fwd_stats": stats_bf16},
        "components_ms": {k_: round(v, 4) for k_, v in comp.items()},
        "kmeanspp_ms": round(ms_kpp, 3),
        "lambda_max": lmax_h,
        "lambda_k_est": lam_k_h,
        "ari_vs_planted": ari_planted,
        "pipeline_normalized": norm_res,
        "pattern_only": None if ms_pat is None else {
            "ms_per_filter_fwd": round(ms_pat, 4), "gbs": round(p * bs_pat / (ms_pat * 1e-3) / 1e9, 2)},
        "roofline": {"bound": "hbm", "achieved": round(alg_launch / (launch_ms * 1e-3) / 1e9, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(alg_launch / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "traffic_kind": "L2-to-fabric bytes per launch (FETCH_SIZE x2 + WRITE_SIZE x1), "
                                     "Infinity Cache hits included",
                     "kernel": "cheb_step", "slice_cols": rs32, "variant": var32,
                     "algorithmic_bytes_per_launch": round(alg_launch), "launch_ms": round(launch_ms, 5),
                     "achieved_y_as_moved": round(alg_launch_ymoved / (launch_ms * 1e-3) / 1e9, 2),
                     "frac_y_as_moved": round(alg_launch_ymoved / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "launches_per_filter": launches,
                     "amplification": None if traffic is None else round(traffic / alg_launch, 3),
                     "traffic_gbs": None if traffic is None else round(traffic / (launch_ms * 1e-3) / 1e9, 1),
                     "copy_gbs_4GiB": round(copy_big["GBps"], 1), "copy_gbs_64MiB": round(copy_llc["GBps"], 1),
                     "frac_of_copy": round(alg_launch / (launch_ms * 1e-3) / 1e9 / (copy_big["GBps"]), 4),
                     "gather_floor_ms": None if gfloor is None else round(gfloor, 5),
                     "frac_of_gather_floor": None if gfloor is None else round(gfloor / launch_ms, 4)},
        "cpu_baseline": cpu,
        "block_order": blk,
        "sbm_n1e3": small_res,
        "sbm_n1e5": mid_res,
        "batch": batch_res,
        "knn_grad": knn_res,
        "stability": stab_res,
        "health": {"flags": health,
                   "ok": all((f & (asc._abi.ASC_FLAG_GROWTH | asc._abi.ASC_FLAG_NONFINITE)) == 0
                             for f in health.values())},
        "extra": extra,
        "gen_s": round(gen_s, 1),
        "software": {"hip": torch.version.hip, "torch": torch.__version__, "device": torch.cuda.get_device_name(0)},
    }
    print(json.dumps(line))
    if not line["health"]["ok"]:
        _progress(f"health flags raised: {health}")
        sys.exit(3)


if __name__ == "__main__":
    main()
