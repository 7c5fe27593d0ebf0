"""The filter and the one-pass lambda_k + filter entry points enqueue no
host synchronisation and no memset, so a caller can capture them in a HIP
graph: every replay must reproduce the eager result exactly."""
import numpy as np
import pytest
import torch

import workloads as W
import paper_1509_08863_amd as asc

from gpu_util import DEV, upload_graph, block_f32, scalar, host, to_dev

pytestmark = pytest.mark.gpu


def test_captured_filter_replays_match_eager():
    g = W.workload_graph(1)
    G = upload_graph(g)
    Rs, _ = W.signals(g.n, 32, 21)
    R = block_f32(Rs)
    lmax = asc.lmax_estimate(G, to_dev(W.start_vector(g.n, 1)), 60)
    a = asc.cheb_coeffs(0.05 * lmax, lmax, 50)
    Y = torch.empty(g.n, 32, dtype=torch.float32, device=DEV)
    ws = asc.workspace(asc._abi.lib().asc_filter_workspace(g.n, 32, asc.ASC_F32, 50), DEV)
    asc.cheb_filter(G, lmax, a, R, Y, ws)
    eager = host(Y).copy()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            asc.cheb_filter(G, lmax, a, R, Y, ws)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        Y.zero_()
        asc.normalize_features(block_f32(np.ones((10, 4), np.float32)))  # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(Y), eager, err_msg=f"replay {rep}")


def test_captured_lambda_k_filter_replays_match_eager():
    g = W.workload_graph(1)
    G = upload_graph(g)
    Rs, _ = W.signals(g.n, 32, 22)
    R = block_f32(Rs)
    lmax = scalar(1.01 * 2 * float(host(G.strength).max()))
    k, p, steps = 10, 50, 12
    Y = torch.empty(g.n, 32, dtype=torch.float32, device=DEV)
    states = asc.workspace(asc._abi.lib().asc_ckpt_bytes(G.c(), 32, asc.ASC_F32, p, 1), DEV)
    _, lam, traj, co, _ = asc.lambda_k_filter(G, lmax, k, p, steps, R, Y, states)
    eager = (host(Y).copy(), host(lam).copy(), host(traj).copy())
    ws = asc.lambda_k_filter.last_ws
    L = asc._abi.lib()
    lam2 = torch.empty(1, dtype=torch.float64, device=DEV)
    traj2 = torch.empty(steps, 2, dtype=torch.float64, device=DEV)
    co2 = torch.empty(p + 1, dtype=torch.float64, device=DEV)

    def run():
        asc._abi.check(L.asc_lambda_k_filter(G.c(), asc._ptr(lmax), k, p, steps, asc._ptr(R), asc.ASC_F32, 32,
                                             R.stride(0), asc._ptr(Y), Y.stride(0), asc._ptr(lam2), asc._ptr(traj2),
                                             asc._ptr(co2), asc._ptr(states), asc._ptr(ws), ws.numel(), asc._stream()))

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            run()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        Y.zero_()
        lam2.zero_()
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(Y), eager[0], err_msg=f"replay {rep}")
        np.testing.assert_array_equal(host(lam2), eager[1])
        np.testing.assert_array_equal(host(traj2), eager[2])
