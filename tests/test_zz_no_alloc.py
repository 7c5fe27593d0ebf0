"""asc_cheb_filter_noalloc (the filter with its workspace in the library's
static device array) against asc_cheb_filter, called through the raw C ABI:
two calls in a row, the second on a smaller graph and block, each equal to the
workspace entry point's result bit for bit and to the float64 oracle within
the float32 bound (1e-5 relative Frobenius); sizes beyond the array are
rejected before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_1509_08863_amd as asc
from paper_1509_08863_amd import _abi

from gpu_util import DEV, block_f32, block_bf16, to_dev, upload_graph

pytestmark = pytest.mark.gpu


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _raw_filter(G, lm, a, R, Y, dt, ws=None):
    L = _abi.lib()
    n, r = R.shape
    p = a.numel() - 1
    if ws is None:
        return L.asc_cheb_filter_noalloc(G.c(), _p(lm), _p(a), p, _p(R), dt, r, R.stride(0), _p(Y), Y.stride(0),
                                         None, 0, _stream())
    return L.asc_cheb_filter(G.c(), _p(lm), _p(a), p, _p(R), dt, r, R.stride(0), _p(Y), Y.stride(0), None, 0,
                             _p(ws), ws.numel(), _stream())


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_noalloc_matches_workspace_filter_twice(dtype):
    cases = [(W.sbm(W.equal_sizes(20000, 8), 16.0, 0.1, 71), 48, 60),   # first call: larger
             (W.sbm(W.equal_sizes(3000, 5), 12.0, 0.1, 72), 17, 30)]    # second call: smaller, ragged r
    for q, (g, r, p) in enumerate(cases):
        print(f"[noalloc] call {q}: {dtype} n={g.n} nnz={g.nnz} r={r} p={p}", flush=True)
        G = upload_graph(g, unit_as_null=True)
        L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, None)
        s = oracle.strength(g.n, g.row_ptr, g.col_idx, None)
        lmax = oracle.lmax_estimate(L, s, W.start_vector(g.n, 73 + q), 40)
        a = oracle.cheb_coeffs(0.2 * lmax, lmax, p)
        if dtype == "f32":
            Rs, R64 = W.signals(g.n, r, 74 + q)
            R, dt = block_f32(Rs), asc.ASC_F32
        else:
            Rs, R64 = W.signals(g.n, r, 74 + q, "bf16")
            R, dt = block_bf16(Rs), asc.ASC_BF16
        lm = to_dev(np.array([lmax]))
        ad = to_dev(a)
        ldy = (r + 3) // 4 * 4
        Y0 = torch.full((g.n, ldy), np.nan, dtype=torch.float32, device=DEV)[:, :r]
        Y1 = torch.full((g.n, ldy), np.nan, dtype=torch.float32, device=DEV)[:, :r]
        ws = asc.workspace(_abi.lib().asc_filter_workspace(g.n, r, dt, p), DEV)
        assert _raw_filter(G, lm, ad, R, Y0, dt, ws) == _abi.ASC_OK, _abi.lib().asc_last_error()
        assert _raw_filter(G, lm, ad, R, Y1, dt) == _abi.ASC_OK, _abi.lib().asc_last_error()
        torch.cuda.synchronize()
        y0, y1 = Y0.cpu().numpy(), Y1.cpu().numpy()
        assert np.array_equal(y0, y1)
        Yref = oracle.cheb_filter(L, lmax, a, R64)
        err = np.linalg.norm(y1 - Yref) / np.linalg.norm(Yref)
        print(f"[noalloc] call {q}: rel err vs float64 {err:.3e}", flush=True)
        assert err <= (1e-5 if dtype == "f32" else 6e-2)


def test_noalloc_rejects_beyond_the_array():
    g = W.cycle(200_000)
    G = upload_graph(g, unit_as_null=True)
    r, p = 96, 10
    need = _abi.lib().asc_filter_workspace(g.n, r, asc.ASC_F32, p)
    assert need > (64 << 20)
    R = torch.zeros(g.n, r, dtype=torch.float32, device=DEV)
    Y = torch.zeros(g.n, r, dtype=torch.float32, device=DEV)
    lm = to_dev(np.array([4.0]))
    a = to_dev(np.ones(p + 1))
    st = _raw_filter(G, lm, a, R, Y, asc.ASC_F32)
    assert st == _abi.ASC_ERR_WORKSPACE
    assert b"static array" in _abi.lib().asc_last_error()
