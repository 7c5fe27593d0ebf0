"""Accelerated spectral clustering by graph filtering of random signals
(Tremblay et al., ICASSP 2016) on MI355X: Python binding of libasc.

Thin argument marshalling over the C ABI of include/asc.h: every function has
the name of its C entry point without the ``asc_`` prefix, takes torch tensors
on the GPU, allocates outputs and workspaces with torch (device memory and
streams are torch's; all arithmetic runs in the HIP kernels) and enqueues the
work on torch's current stream.
"""
from __future__ import annotations

import ctypes

import torch

from . import _abi
from ._abi import AscError, ASC_F32, ASC_BF16  # noqa: F401

__all__ = ["Graph", "graph_prepare", "lmax_estimate", "cheb_coeffs", "cheb_filter", "cheb_moments",
           "eigcount_dichotomy", "eigcount_lambda_k", "normalize_features", "kmeans_init_rows",
           "kmeans_assign", "kmeans_update", "kmeans_replicates", "read_flags", "workspace", "AscError", "tune_set", "tune_get",
           "tune_save", "tune_load", "autotune_filter", "cheb_filter_bwd", "gauss_weights", "gauss_weights_bwd",
           "rownorm_loss_bwd", "Batch", "stream_copy",
           "lambda_k_filter", "cheb_filter_noalloc"]


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return ASC_F32
    if t.dtype == torch.bfloat16:
        return ASC_BF16
    raise TypeError(f"signal block must be float32 or bfloat16, got {t.dtype}")


def _ld(t: torch.Tensor) -> int:
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("blocks must be 2-D with unit column stride")
    return t.stride(0)


def workspace(nbytes: int, device) -> torch.Tensor:
    """A 256-byte aligned device buffer of at least nbytes (torch-allocated)."""
    buf = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + max(int(nbytes), 1)]


class Graph:
    """CSR graph W on the device plus its float64 strengths (asc_graph)."""

    def __init__(self, row_ptr: torch.Tensor, col_idx: torch.Tensor, w: torch.Tensor | None,
                 strength: torch.Tensor):
        self.row_ptr, self.col_idx, self.w, self.strength = row_ptr, col_idx, w, strength
        self.n = row_ptr.numel() - 1
        self.nnz = col_idx.numel()
        self._c = _abi.asc_graph(self.n, self.nnz, row_ptr.data_ptr(), col_idx.data_ptr() if self.nnz else None,
                                 None if w is None else w.data_ptr(), strength.data_ptr())

    @property
    def device(self):
        return self.row_ptr.device

    def c(self):
        return ctypes.byref(self._c)

    def with_weights(self, w: torch.Tensor | None) -> "Graph":
        """Same pattern with other weights (strengths must be re-prepared)."""
        return graph_prepare(self.row_ptr, self.col_idx, w)


def graph_prepare(row_ptr: torch.Tensor, col_idx: torch.Tensor, w: torch.Tensor | None = None,
                  validate: bool = False) -> Graph:
    L = _abi.lib()
    n = row_ptr.numel() - 1
    strength = torch.empty(n, dtype=torch.float64, device=row_ptr.device)
    g = Graph(row_ptr, col_idx, w, strength)
    ws = workspace(L.asc_graph_prepare_workspace(n, int(validate)), row_ptr.device) if validate else None
    _abi.check(L.asc_graph_prepare(g.c(), _ptr(strength), int(validate), _ptr(ws),
                                   0 if ws is None else ws.numel(), _stream()))
    return g


def graph_normalized(g: Graph) -> Graph:
    """The same pattern with w_e / sqrt(s_i s_k) and unit strengths: entry
    points called on it apply L_n = I - S^-1/2 W S^-1/2 (lmax = 2 is valid)."""
    wn = torch.empty(max(g.nnz, 1), dtype=torch.float32, device=g.device)[:g.nnz]
    ones = torch.empty(g.n, dtype=torch.float64, device=g.device)
    _abi.check(_abi.lib().asc_graph_normalize(g.c(), _ptr(wn) if g.nnz else None, _ptr(ones), _stream()))
    return Graph(g.row_ptr, g.col_idx, wn, ones)


def lmax_estimate(g: Graph, v0: torch.Tensor, iters: int = 60, host: bool = False):
    L = _abi.lib()
    out = torch.empty(1, dtype=torch.float64, device=g.device)
    ws = workspace(L.asc_lmax_workspace(g.n, iters), g.device)
    h = ctypes.c_double(0.0)
    _abi.check(L.asc_lmax_estimate(g.c(), _ptr(v0), iters, _ptr(out), ctypes.byref(h) if host else None,
                                   _ptr(ws), ws.numel(), _stream()))
    return (out, h.value) if host else out


def cheb_coeffs(lambda_c: torch.Tensor, lmax: torch.Tensor, p: int, jackson: bool = True) -> torch.Tensor:
    lambda_c = lambda_c.reshape(-1)
    out = torch.empty(lambda_c.numel(), p + 1, dtype=torch.float64, device=lambda_c.device)
    _abi.check(_abi.lib().asc_cheb_coeffs(_ptr(lambda_c), lambda_c.numel(), _ptr(lmax), p, int(jackson),
                                          _ptr(out), _stream()))
    return out


def cheb_filter(g: Graph, lmax: torch.Tensor, coeffs: torch.Tensor, R: torch.Tensor, Y: torch.Tensor | None = None,
                ws: torch.Tensor | None = None, ckpt_stride: int = 0, ckpt: torch.Tensor | None = None):
    """Y = sum_j a_j T_j(Lt) R.  With ckpt_stride >= 2 also returns the
    checkpoint buffer that cheb_filter_bwd needs: (Y, ckpt)."""
    L = _abi.lib()
    coeffs = coeffs.reshape(-1)
    p = coeffs.numel() - 1
    n, r = R.shape
    if Y is None:
        ldy = (r + 3) // 4 * 4
        Y = torch.empty(n, ldy, dtype=torch.float32, device=R.device)[:, :r]
    dt = _dtype_code(R)
    need = L.asc_filter_workspace(n, r, dt, p)
    if ws is None or ws.numel() < need:
        ws = workspace(need, R.device)
    ck = None
    if ckpt_stride:
        need_ck = L.asc_ckpt_bytes(g.c(), r, dt, p, ckpt_stride)
        ck = ckpt if (ckpt is not None and ckpt.numel() >= need_ck) else workspace(need_ck, R.device)
    _abi.check(L.asc_cheb_filter(g.c(), _ptr(lmax), _ptr(coeffs), p, _ptr(R), dt, r, _ld(R), _ptr(Y), _ld(Y),
                                 _ptr(ck), ckpt_stride, _ptr(ws), ws.numel(), _stream()))
    cheb_filter.last_ws = ws
    return (Y, ck) if ckpt_stride else Y


def cheb_filter_noalloc(g: Graph, lmax: torch.Tensor, coeffs: torch.Tensor, R: torch.Tensor, Y: torch.Tensor,
                       ckpt: torch.Tensor | None = None, ckpt_stride: int = 0) -> torch.Tensor:
    """cheb_filter into the caller's Y with the library's static device
    scratch as workspace (asc_cheb_filter_noalloc): allocates nothing."""
    coeffs = coeffs.reshape(-1)
    n, r = R.shape
    _abi.check(_abi.lib().asc_cheb_filter_noalloc(g.c(), _ptr(lmax), _ptr(coeffs), coeffs.numel() - 1, _ptr(R),
                                                  _dtype_code(R), r, _ld(R), _ptr(Y), _ld(Y), _ptr(ckpt),
                                                  ckpt_stride, _stream()))
    return Y


def cheb_filter_bwd(g: Graph, lmax: torch.Tensor, coeffs: torch.Tensor, R: torch.Tensor, ckpt: torch.Tensor,
                    ckpt_stride: int, G: torch.Tensor, want_dw: bool = True, want_dcoeffs: bool = True,
                    ws: torch.Tensor | None = None):
    """(dW per stored entry float32 or None, dcoeffs float64 or None)."""
    L = _abi.lib()
    coeffs = coeffs.reshape(-1)
    p = coeffs.numel() - 1
    n, r = R.shape
    dt = _dtype_code(R)
    dW = torch.empty(g.nnz, dtype=torch.float32, device=R.device) if want_dw else None
    dc = torch.empty(p + 1, dtype=torch.float64, device=R.device) if want_dcoeffs else None
    need = L.asc_filter_bwd_workspace(n, g.nnz, r, dt, p, ckpt_stride)
    if ws is None or ws.numel() < need:
        ws = workspace(need, R.device)
    cheb_filter_bwd.last_ws = ws
    _abi.check(L.asc_cheb_filter_bwd(g.c(), _ptr(lmax), _ptr(coeffs), p, _ptr(R), dt, r, _ld(R), _ptr(ckpt),
                                     ckpt_stride, _ptr(G), _ld(G), _ptr(dW), _ptr(dc), _ptr(ws), ws.numel(),
                                     _stream()))
    return dW, dc


def gauss_weights(d2: torch.Tensor, sigma: float) -> torch.Tensor:
    w = torch.empty_like(d2)
    _abi.check(_abi.lib().asc_gauss_weights(_ptr(d2), d2.numel(), float(sigma), _ptr(w), _stream()))
    return w


def gauss_weights_bwd(d2: torch.Tensor, w: torch.Tensor, dW: torch.Tensor, sigma: float) -> torch.Tensor:
    L = _abi.lib()
    out = torch.empty(1, dtype=torch.float64, device=d2.device)
    ws = workspace(L.asc_gauss_weights_bwd_workspace(d2.numel()), d2.device)
    _abi.check(L.asc_gauss_weights_bwd(_ptr(d2), _ptr(w), _ptr(dW), d2.numel(), float(sigma), _ptr(out), _ptr(ws),
                                       ws.numel(), _stream()))
    return out


def rownorm_loss_bwd(Y: torch.Tensor, target: torch.Tensor):
    """(loss float64 [1], G = dloss/dY float32) for loss = sum_i |y_i/|y_i| - t_i|^2."""
    L = _abi.lib()
    n, r = Y.shape
    loss = torch.empty(1, dtype=torch.float64, device=Y.device)
    G = torch.empty(n, (r + 3) // 4 * 4, dtype=torch.float32, device=Y.device)[:, :r]
    ws = workspace(L.asc_rownorm_loss_bwd_workspace(n), Y.device)
    _abi.check(L.asc_rownorm_loss_bwd(_ptr(Y), _ld(Y), _ptr(target), _ld(target), n, r, _ptr(loss), _ptr(G), _ld(G),
                                      _ptr(ws), ws.numel(), _stream()))
    return loss, G


def cheb_moments(g: Graph, lmax: torch.Tensor, p: int, R: torch.Tensor) -> torch.Tensor:
    L = _abi.lib()
    n, r = R.shape
    dt = _dtype_code(R)
    mu = torch.empty(p + 1, dtype=torch.float64, device=R.device)
    ws = workspace(L.asc_moments_workspace(n, r, dt, p), R.device)
    _abi.check(L.asc_cheb_moments(g.c(), _ptr(lmax), p, _ptr(R), dt, r, _ld(R), _ptr(mu), _ptr(ws), ws.numel(),
                                  _stream()))
    cheb_moments.last_ws = ws
    return mu


def eigcount_dichotomy(mu: torch.Tensor, lmax: torch.Tensor, k: int, steps: int, jackson: bool = True):
    lam = torch.empty(1, dtype=torch.float64, device=mu.device)
    traj = torch.empty(max(steps, 1), 2, dtype=torch.float64, device=mu.device)
    _abi.check(_abi.lib().asc_eigcount_dichotomy(_ptr(mu), mu.numel() - 1, _ptr(lmax), k, steps, int(jackson),
                                                 _ptr(lam), _ptr(traj), _stream()))
    return lam, traj[:steps]


def eigcount_lambda_k(g: Graph, lmax: torch.Tensor, k: int, p: int, steps: int, R: torch.Tensor,
                      literal: bool = False):
    L = _abi.lib()
    n, r = R.shape
    dt = _dtype_code(R)
    lam = torch.empty(1, dtype=torch.float64, device=R.device)
    traj = torch.empty(max(steps, 1), 2, dtype=torch.float64, device=R.device)
    ws = workspace(L.asc_eigcount_workspace(n, r, dt, p, steps, int(literal)), R.device)
    _abi.check(L.asc_eigcount_lambda_k(g.c(), _ptr(lmax), k, p, steps, int(literal), _ptr(R), dt, r, _ld(R),
                                       _ptr(lam), _ptr(traj), _ptr(ws), ws.numel(), _stream()))
    eigcount_lambda_k.last_ws = ws
    return lam, traj[:steps]


def lambda_k_filter(g: Graph, lmax: torch.Tensor, k: int, p: int, steps: int, R: torch.Tensor,
                    Y: torch.Tensor | None = None, states: torch.Tensor | None = None):
    """One recurrence pass: (Y, lambda_k, traj, coeffs, states); `states`
    (all T_j R) can be passed to cheb_filter_bwd with ckpt_stride=1."""
    L = _abi.lib()
    n, r = R.shape
    dt = _dtype_code(R)
    if Y is None:
        Y = torch.empty(n, (r + 3) // 4 * 4, dtype=torch.float32, device=R.device)[:, :r]
    need = L.asc_ckpt_bytes(g.c(), r, dt, p, 1)
    if states is None or states.numel() < need:
        states = workspace(need, R.device)
    lam = torch.empty(1, dtype=torch.float64, device=R.device)
    traj = torch.empty(max(steps, 1), 2, dtype=torch.float64, device=R.device)
    co = torch.empty(p + 1, dtype=torch.float64, device=R.device)
    ws = workspace(L.asc_lambda_k_filter_workspace(n, r, dt, p), R.device)
    _abi.check(L.asc_lambda_k_filter(g.c(), _ptr(lmax), k, p, steps, _ptr(R), dt, r, _ld(R), _ptr(Y), _ld(Y),
                                     _ptr(lam), _ptr(traj), _ptr(co), _ptr(states), _ptr(ws), ws.numel(), _stream()))
    lambda_k_filter.last_ws = ws
    return Y, lam, traj[:steps], co, states


def normalize_features(Y: torch.Tensor, want_norms: bool = True):
    n, r = Y.shape
    norms = torch.empty(n, dtype=torch.float32, device=Y.device) if want_norms else None
    _abi.check(_abi.lib().asc_normalize_features(_ptr(Y), n, r, _ld(Y), _ptr(norms), _stream()))
    return norms


def kmeans_init_rows(F: torch.Tensor, rows: torch.Tensor) -> torch.Tensor:
    n, r = F.shape
    k = rows.numel()
    C = torch.empty(k, r, dtype=torch.float32, device=F.device)
    _abi.check(_abi.lib().asc_kmeans_init_rows(_ptr(F), n, r, _ld(F), _ptr(rows), k, _ptr(C), _stream()))
    return C


def kmeans_assign(F: torch.Tensor, C: torch.Tensor, dist: bool = True):
    """(labels, dist2); dist=False returns (labels, None) and lets the library
    skip the float64 distance of rows whose nearest centroid is already certain."""
    n, r = F.shape
    k = C.shape[0]
    labels = torch.empty(n, dtype=torch.int32, device=F.device)
    dist2 = torch.empty(n, dtype=torch.float32, device=F.device) if dist else None
    _abi.check(_abi.lib().asc_kmeans_assign(_ptr(F), n, r, _ld(F), _ptr(C.contiguous()), k, _ptr(labels),
                                            _ptr(dist2), _stream()))
    return labels, dist2


def kmeans_pp(F: torch.Tensor, k: int, U: torch.Tensor) -> torch.Tensor:
    """Rows (int32 device tensor, k) chosen by the k-means++ draw with the
    caller's 53-bit random integers U (int64 or uint64 tensor of k values)."""
    L = _abi.lib()
    n, r = F.shape
    U = U.to(F.device).contiguous()
    rows = torch.empty(k, dtype=torch.int32, device=F.device)
    ws = workspace(L.asc_kmeanspp_workspace(n), F.device)
    _abi.check(L.asc_kmeanspp(_ptr(F), n, r, _ld(F), k, _ptr(U), _ptr(rows), _ptr(ws), ws.numel(), _stream()))
    kmeans_pp.last_ws = ws
    return rows


def kmeans_update(F: torch.Tensor, labels: torch.Tensor, C: torch.Tensor, ws: torch.Tensor | None = None):
    """Updates C (k x r float32, contiguous) in place; returns the member counts."""
    L = _abi.lib()
    n, r = F.shape
    k = C.shape[0]
    assert C.is_contiguous()
    counts = torch.empty(k, dtype=torch.int64, device=F.device)
    need = L.asc_kmeans_update_workspace(n, r, k)
    if ws is None or ws.numel() < need:
        ws = workspace(need, F.device)
    _abi.check(L.asc_kmeans_update(_ptr(F), n, r, _ld(F), _ptr(labels), k, _ptr(C), _ptr(counts), _ptr(ws),
                                   ws.numel(), _stream()))
    return counts


def kmeans_replicates(F: torch.Tensor, rows: torch.Tensor, iters: int):
    """Lloyd's method from each row of `rows` (reps x k tensor of initial rows
    of F), iters steps each; returns (labels, C, inertia): the labels and
    centroids of the run of least inertia and every run's inertia (float64)."""
    L = _abi.lib()
    n, r = F.shape
    reps, k = rows.shape
    rows = rows.to(device=F.device, dtype=torch.int32).contiguous()
    labels = torch.empty(n, dtype=torch.int32, device=F.device)
    C = torch.empty(k, r, dtype=torch.float32, device=F.device)
    inertia = torch.empty(reps, dtype=torch.float64, device=F.device)
    ws = workspace(L.asc_kmeans_replicates_workspace(n, r, k, reps), F.device)
    _abi.check(L.asc_kmeans_replicates(_ptr(F), n, r, _ld(F), k, reps, iters, _ptr(rows), _ptr(labels), _ptr(C),
                                       _ptr(inertia), _ptr(ws), ws.numel(), _stream()))
    kmeans_replicates.last_ws = ws
    return labels, C, inertia


def read_flags(ws: torch.Tensor, raise_on_error: bool = True) -> int:
    f = ctypes.c_uint32(0)
    st = _abi.lib().asc_read_flags(_ptr(ws), ctypes.byref(f), _stream())
    if raise_on_error:
        _abi.check(st)
    return int(f.value)


def tune_set(g: Graph, r: int, dtype: torch.dtype, slice_cols: int, variant: int = 0) -> None:
    dt = ASC_F32 if dtype == torch.float32 else ASC_BF16
    _abi.check(_abi.lib().asc_tune_set(g.n, g.nnz, r, dt, slice_cols, variant))


def tune_get(g: Graph, r: int, dtype: torch.dtype):
    dt = ASC_F32 if dtype == torch.float32 else ASC_BF16
    rs, var = ctypes.c_int(0), ctypes.c_int(0)
    _abi.check(_abi.lib().asc_tune_get(g.n, g.nnz, r, dt, ctypes.byref(rs), ctypes.byref(var)))
    return rs.value, var.value


def tune_save(path: str) -> None:
    _abi.check(_abi.lib().asc_tune_save(path.encode()))


def tune_load(path: str) -> None:
    _abi.check(_abi.lib().asc_tune_load(path.encode()))


def autotune_filter(g: Graph, lmax: torch.Tensor, R: torch.Tensor, probe_steps: int = 3):
    """Times every (slice width, variant) candidate; returns (slice_cols, variant, ms per step)."""
    L = _abi.lib()
    n, r = R.shape
    dt = _dtype_code(R)
    Y = torch.empty(n, (r + 3) // 4 * 4, dtype=torch.float32, device=R.device)[:, :r]
    ws = workspace(L.asc_filter_workspace(n, r, dt, 1), R.device)
    rs, var, ms = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_float(0)
    _abi.check(L.asc_autotune_filter(g.c(), _ptr(lmax), _ptr(R), dt, r, _ld(R), _ptr(Y), _ld(Y), probe_steps,
                                     _ptr(ws), ws.numel(), ctypes.byref(rs), ctypes.byref(var), ctypes.byref(ms),
                                     _stream()))
    return rs.value, var.value, ms.value


class Batch:
    """Batched lambda_k estimation + filtering of a block-diagonal graph
    (asc_batch_*): graph q owns rows node_off[q]..node_off[q+1]-1."""

    def __init__(self, g: Graph, node_off, k, r: int, dtype: torch.dtype, p: int, steps: int, tile_rows: int = 0):
        import numpy as np
        L = _abi.lib()
        self._off = np.ascontiguousarray(node_off, dtype=np.int64)
        self._k = np.ascontiguousarray(k, dtype=np.int32)
        self.G = len(self._k)
        self.g, self.r, self.p, self.steps = g, r, p, steps
        self.dt = ASC_F32 if dtype == torch.float32 else ASC_BF16
        h = ctypes.c_void_p(None)
        _abi.check(L.asc_batch_create(g.c(), self.G, self._off.ctypes.data, self._k.ctypes.data, r, self.dt, p,
                                      steps, tile_rows, ctypes.byref(h)))
        self._h = h
        self.ws = workspace(L.asc_batch_workspace(h), g.device)

    def info(self):
        a, b, c = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        _abi.check(_abi.lib().asc_batch_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"slice_cols": a.value, "tile_rows": b.value, "ntiles": c.value}

    def run(self, lmax: torch.Tensor, R: torch.Tensor, Y: torch.Tensor, lambda_k: torch.Tensor,
            traj: torch.Tensor | None = None, use_graph: bool = True) -> None:
        _abi.check(_abi.lib().asc_batch_run(self._h, _ptr(lmax), _ptr(R), _ld(R), _ptr(Y), _ld(Y), _ptr(lambda_k),
                                            _ptr(traj), _ptr(self.ws), self.ws.numel(), int(use_graph), _stream()))

    def autotune(self, lmax: torch.Tensor, R: torch.Tensor, Y: torch.Tensor, lambda_k: torch.Tensor,
                 traj: torch.Tensor | None = None, probe_runs: int = 1):
        """Times the candidate slice widths x tile sizes on this batch
        (asc_batch_autotune), re-plans with the fastest and resizes the
        workspace; Y, lambda_k and traj are scratch."""
        L = _abi.lib()
        ws = workspace(L.asc_batch_tune_workspace(self._h), self.g.device)
        a, b, c = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_float(0.0)
        _abi.check(L.asc_batch_autotune(self._h, _ptr(lmax), _ptr(R), _ld(R), _ptr(Y), _ld(Y), _ptr(lambda_k),
                                        _ptr(traj), probe_runs, _ptr(ws), ws.numel(), ctypes.byref(a),
                                        ctypes.byref(b), ctypes.byref(c), _stream()))
        del ws
        self.ws = workspace(L.asc_batch_workspace(self._h), self.g.device)
        return {"slice_cols": a.value, "tile_rows": b.value, "ms": c.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _abi.lib().asc_batch_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stability(g: Graph, lmax: torch.Tensor, k_min: int, k_max: int, etas, J: int, reps: int, p: int, steps: int,
              kmeans_iters: int, R: torch.Tensor, eta_max: int, init_rows: torch.Tensor, ws: torch.Tensor | None = None):
    """Stability measure gamma(k), k = k_min..k_max (Eq. stab).  R is n x (J *
    eta_max) unit-variance columns (realisation j = columns j*eta_max ...);
    init_rows int32 [nk][J][reps][k_max].  Returns a dict of device tensors:
    gamma [nk], ari [nk][J(J-1)/2], labels [nk][J][n], lambda_k [nk][J],
    traj [nk][J][steps][2], inertia [nk][J][reps]."""
    L = _abi.lib()
    n = R.shape[0]
    nk = k_max - k_min + 1
    eta_arr = (ctypes.c_int * nk)(*[int(e) for e in etas])
    dt = _dtype_code(R)
    need = L.asc_stability_workspace(g.c(), k_min, k_max, eta_arr, J, reps, p, steps, dt, eta_max)
    if need == 0:
        raise _abi.AscError(_abi.ASC_ERR_INVALID, L.asc_last_error().decode())
    if ws is None or ws.numel() < need:
        ws = workspace(need, R.device)
    dev = R.device
    npairs = J * (J - 1) // 2
    out = {
        "gamma": torch.empty(nk, dtype=torch.float64, device=dev),
        "ari": torch.empty(nk, npairs, dtype=torch.float64, device=dev),
        "labels": torch.empty(nk, J, n, dtype=torch.int32, device=dev),
        "lambda_k": torch.empty(nk, J, dtype=torch.float64, device=dev),
        "traj": torch.empty(nk, J, max(steps, 1), 2, dtype=torch.float64, device=dev),
        "inertia": torch.empty(nk, J, reps, dtype=torch.float64, device=dev),
    }
    _abi.check(L.asc_stability(g.c(), _ptr(lmax), k_min, k_max, eta_arr, J, reps, p, steps, kmeans_iters, _ptr(R), dt,
                               eta_max, _ld(R), _ptr(init_rows), _ptr(out["gamma"]), _ptr(out["ari"]),
                               _ptr(out["labels"]), _ptr(out["lambda_k"]), _ptr(out["traj"]), _ptr(out["inertia"]),
                               _ptr(ws), ws.numel(), _stream()))
    out["traj"] = out["traj"][:, :, :steps]
    stability.last_ws = ws
    return out


def knn_graph(X: torch.Tensor, k: int):
    """K-nearest-neighbour graph of the rows of X (float32 n x d, d <= 64):
    returns dict with nbr [n][k] int32, nbr_d2 [n][k] float64 (exact, ties to
    the lower index), row_ptr / col_idx (int32) and d2 (float32) of the
    union-symmetrised graph, and fallback_rows (device uint32)."""
    L = _abi.lib()
    n, d = X.shape
    if X.stride(1) != 1:
        raise ValueError("X must have unit column stride")
    dev = X.device
    ws = workspace(L.asc_knn_workspace(n, d, k), dev)
    nbr = torch.empty(n, k, dtype=torch.int32, device=dev)
    nd2 = torch.empty(n, k, dtype=torch.float64, device=dev)
    row_ptr = torch.empty(n + 1, dtype=torch.int32, device=dev)
    fb = torch.zeros(1, dtype=torch.int32, device=dev)
    _abi.check(L.asc_knn(_ptr(X), n, d, X.stride(0), k, _ptr(nbr), _ptr(nd2), _ptr(row_ptr), _ptr(fb), _ptr(ws),
                         ws.numel(), _stream()))
    nnz = int(row_ptr[n].item())
    col_idx = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)[:nnz]
    d2 = torch.empty(max(nnz, 1), dtype=torch.float32, device=dev)[:nnz]
    _abi.check(L.asc_knn_graph_fill(_ptr(X), n, d, X.stride(0), k, _ptr(nbr), _ptr(row_ptr), _ptr(col_idx), _ptr(d2),
                                    _ptr(ws), ws.numel(), _stream()))
    return {"nbr": nbr, "nbr_d2": nd2, "row_ptr": row_ptr, "col_idx": col_idx, "d2": d2, "fallback_rows": fb}


def order_table(rho: torch.Tensor, delta: torch.Tensor, band: float, m_max: int, grid: int = 2049,
                jackson: bool = True):
    """Least orders m*[q][d] meeting delta[d] outside the band for each
    rho[q] = lambda_c / lambda_N, and the errors err[q][m-1] (device tensors)."""
    rho = rho.to(torch.float64).contiguous()
    delta = delta.to(torch.float64).contiguous()
    err = torch.empty(rho.numel(), m_max, dtype=torch.float64, device=rho.device)
    ms = torch.empty(rho.numel(), delta.numel(), dtype=torch.int32, device=rho.device)
    _abi.check(_abi.lib().asc_order_table(_ptr(rho), rho.numel(), _ptr(delta), delta.numel(), float(band), m_max, grid,
                                          int(jackson), _ptr(err), _ptr(ms), None, 0, _stream()))
    return ms, err


def order_for(lambda_c: float, lmax: float, delta: float = 0.1, band_rel: float = 0.5, m_max: int = 4000,
              grid: int = 2049, device="cuda:0") -> int:
    """Order for one filter: m*(lambda_c / lmax; delta) with the transition
    band set to band_rel * lambda_c (host int)."""
    rho = lambda_c / lmax
    ms, _ = order_table(torch.tensor([rho], dtype=torch.float64, device=device),
                        torch.tensor([delta], dtype=torch.float64, device=device), band_rel * rho, m_max, grid)
    return int(ms.cpu()[0, 0])


def lambda_k_filter_auto(g: Graph, lmax: torch.Tensor, k: int, R: torch.Tensor, delta: float = 0.1,
                         band_rel: float = 0.5, p_count: int = 150, steps: int = 12, m_max: int = 4000,
                         grid: int = 2049, Y: torch.Tensor | None = None):
    """Steps 2-5 of Sec. 4.1 with the polynomial order taken from the order
    table (note on m, Sec. 2.4): lambda_k by the dichotomy on Chebyshev moments
    of order p_count, then p = m*(lambda_k / lmax; delta) with a transition
    band of band_rel * lambda_k, then the order-p filter at lambda_k.  Reads
    lambda_k, lmax and m* back to the host (the order sizes the recurrence).
    Returns (Y, lambda_k, traj, p); raises ValueError if no order up to m_max
    meets delta."""
    lam, traj = eigcount_lambda_k(g, lmax, k, p_count, steps, R)
    lam_h, lmax_h = float(lam.cpu()[0]), float(lmax.reshape(-1)[0].cpu())
    if not 0.0 < lam_h < lmax_h:
        raise ValueError(f"lambda_k = {lam_h} outside (0, lambda_max = {lmax_h}): no low-pass order to choose")
    p = order_for(lam_h, lmax_h, delta, band_rel, m_max, grid, device=R.device)
    if p > m_max:
        raise ValueError(f"no order up to {m_max} meets delta = {delta} outside the band")
    Y = cheb_filter(g, lmax, cheb_coeffs(lam, lmax, p), R, Y)
    return Y, lam, traj, p


def ari_pairs(labels: torch.Tensor, k: int):
    """Adjusted Rand index of every pair (a, b), a < b, of the J labellings in
    the rows of labels (int32 J x n, values in [0, k)); returns (ari, mean)."""
    L = _abi.lib()
    J, n = labels.shape
    ari = torch.empty(J * (J - 1) // 2, dtype=torch.float64, device=labels.device)
    mean = torch.empty(1, dtype=torch.float64, device=labels.device)
    ws = workspace(L.asc_ari_workspace(), labels.device)
    _abi.check(L.asc_ari_pairs(_ptr(labels), n, labels.stride(0), J, k, _ptr(ari), _ptr(mean), _ptr(ws), ws.numel(),
                               _stream()))
    ari_pairs.last_ws = ws
    return ari, mean


def gather_probe(table: torch.Tensor, idx: torch.Tensor, sink: torch.Tensor) -> None:
    """Reads rows idx[e] of a (rows x 32) float32 table (asc_gather_probe)."""
    assert table.dtype == torch.float32 and table.dim() == 2 and table.shape[1] == 32 and table.is_contiguous()
    assert idx.dtype == torch.int32 and idx.is_contiguous()
    _abi.check(_abi.lib().asc_gather_probe(_ptr(table), table.shape[0], _ptr(idx), idx.numel(), _ptr(sink),
                                           _stream()))


def stream_copy(src: torch.Tensor, dst: torch.Tensor) -> None:
    """dst <- src (same byte size), plain 16-byte streaming copy kernel."""
    nb = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nb
    _abi.check(_abi.lib().asc_stream_copy(_ptr(src), _ptr(dst), nb, _stream()))
