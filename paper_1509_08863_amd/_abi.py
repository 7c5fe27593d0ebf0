"""ctypes declarations of libasc.so (include/asc.h).  Loading fails loudly if
the library has not been built: there is no fallback implementation."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# ASC_LIBRARY names another build of the same library (the host-sanitizer
# build the CPU tests use); by default the in-tree libasc.so
LIB_PATH = os.environ.get("ASC_LIBRARY") or os.path.join(HERE, "libasc.so")

ASC_OK = 0
ASC_ERR_INVALID = 1
ASC_ERR_WORKSPACE = 2
ASC_ERR_HIP = 3
ASC_ERR_NONFINITE = 4
ASC_ERR_LMAX_TOO_SMALL = 5
ASC_F32 = 0
ASC_BF16 = 1
ASC_FLAG_NONFINITE = 1
ASC_FLAG_GROWTH = 2
ASC_FLAG_BAD_GRAPH = 4
ASC_FLAG_BAD_INPUT = 8

STATUS_NAMES = {0: "ASC_OK", 1: "ASC_ERR_INVALID", 2: "ASC_ERR_WORKSPACE", 3: "ASC_ERR_HIP",
                4: "ASC_ERR_NONFINITE", 5: "ASC_ERR_LMAX_TOO_SMALL"}


class AscError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class asc_graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("w", ctypes.c_void_p), ("strength", ctypes.c_void_p)]


P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int
D = ctypes.c_double
SZ = ctypes.c_size_t
GP = ctypes.POINTER(asc_graph)

# name -> (restype, argtypes); one line per entry point of include/asc.h
SIGNATURES = {
    "asc_abi_version": (ctypes.c_int, []),
    "asc_last_error": (ctypes.c_char_p, []),
    "asc_graph_prepare_workspace": (SZ, [I64, I32]),
    "asc_graph_prepare": (I32, [GP, P, I32, P, SZ, P]),
    "asc_lmax_workspace": (SZ, [I64, I32]),
    "asc_lmax_estimate": (I32, [GP, P, I32, P, P, P, SZ, P]),
    "asc_cheb_coeffs": (I32, [P, I32, P, I32, I32, P, P]),
    "asc_filter_workspace": (SZ, [I64, I64, I32, I32]),
    "asc_ckpt_bytes": (SZ, [GP, I64, I32, I32, I32]),
    "asc_lambda_k_filter_workspace": (SZ, [I64, I64, I32, I32]),
    "asc_lambda_k_filter": (I32, [GP, P, I32, I32, I32, P, I32, I64, I64, P, I64, P, P, P, P, P, SZ, P]),
    "asc_cheb_filter": (I32, [GP, P, P, I32, P, I32, I64, I64, P, I64, P, I32, P, SZ, P]),
    "asc_cheb_filter_noalloc": (I32, [GP, P, P, I32, P, I32, I64, I64, P, I64, P, I32, P]),
    "asc_moments_workspace": (SZ, [I64, I64, I32, I32]),
    "asc_cheb_moments": (I32, [GP, P, I32, P, I32, I64, I64, P, P, SZ, P]),
    "asc_eigcount_dichotomy": (I32, [P, I32, P, I32, I32, I32, P, P, P]),
    "asc_eigcount_workspace": (SZ, [I64, I64, I32, I32, I32, I32]),
    "asc_eigcount_lambda_k": (I32, [GP, P, I32, I32, I32, I32, P, I32, I64, I64, P, P, P, SZ, P]),
    "asc_normalize_features": (I32, [P, I64, I64, I64, P, P]),
    "asc_kmeans_init_rows": (I32, [P, I64, I64, I64, P, I32, P, P]),
    "asc_kmeans_assign": (I32, [P, I64, I64, I64, P, I32, P, P, P]),
    "asc_kmeans_update_workspace": (SZ, [I64, I64, I32]),
    "asc_kmeanspp_workspace": (SZ, [I64]),
    "asc_kmeanspp": (I32, [P, I64, I64, I64, I32, P, P, P, SZ, P]),
    "asc_kmeans_update": (I32, [P, I64, I64, I64, P, I32, P, P, P, SZ, P]),
    "asc_kmeans_replicates_workspace": (SZ, [I64, I64, I32, I32]),
    "asc_kmeans_replicates": (I32, [P, I64, I64, I64, I32, I32, I32, P, P, P, P, P, SZ, P]),
    "asc_stream_copy": (I32, [P, P, SZ, P]),
    "asc_gather_probe": (I32, [P, I64, P, I64, P, P]),
    "asc_read_flags": (I32, [P, ctypes.POINTER(ctypes.c_uint32), P]),
    "asc_gauss_weights": (I32, [P, I64, D, P, P]),
    "asc_gauss_weights_bwd_workspace": (SZ, [I64]),
    "asc_gauss_weights_bwd": (I32, [P, P, P, I64, D, P, P, SZ, P]),
    "asc_rownorm_loss_bwd_workspace": (SZ, [I64]),
    "asc_rownorm_loss_bwd": (I32, [P, I64, P, I64, I64, I64, P, P, I64, P, SZ, P]),
    "asc_filter_bwd_workspace": (SZ, [I64, I64, I64, I32, I32, I32]),
    "asc_cheb_filter_bwd": (I32, [GP, P, P, I32, P, I32, I64, I64, P, I32, P, I64, P, P, P, SZ, P]),
    "asc_batch_create": (I32, [GP, I32, P, P, I64, I32, I32, I32, I32, ctypes.POINTER(ctypes.c_void_p)]),
    "asc_batch_workspace": (SZ, [P]),
    "asc_batch_info": (I32, [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                             ctypes.POINTER(ctypes.c_int)]),
    "asc_batch_run": (I32, [P, P, P, I64, P, I64, P, P, P, SZ, I32, P]),
    "asc_batch_destroy": (I32, [P]),
    "asc_batch_tune_workspace": (SZ, [P]),
    "asc_batch_autotune": (I32, [P, P, P, I64, P, I64, P, P, I32, P, SZ, ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float), P]),
    "asc_graph_normalize": (I32, [GP, P, P, P]),
    "asc_knn_workspace": (SZ, [I64, I32, I32]),
    "asc_knn": (I32, [P, I64, I32, I64, I32, P, P, P, P, P, SZ, P]),
    "asc_knn_graph_fill": (I32, [P, I64, I32, I64, I32, P, P, P, P, P, SZ, P]),
    "asc_order_table_workspace": (SZ, [I32, I32]),
    "asc_order_table": (I32, [P, I32, P, I32, D, I32, I32, I32, P, P, P, SZ, P]),
    "asc_stability_workspace": (SZ, [GP, I32, I32, P, I32, I32, I32, I32, I32, I64]),
    "asc_stability": (I32, [GP, P, I32, I32, P, I32, I32, I32, I32, I32, P, I32, I64, I64, P, P, P, P, P, P, P, P,
                            SZ, P]),
    "asc_ari_workspace": (SZ, []),
    "asc_ari_pairs": (I32, [P, I64, I64, I32, I32, P, P, P, SZ, P]),
    "asc_tune_set": (I32, [I64, I64, I64, I32, I32, I32]),
    "asc_tune_get": (I32, [I64, I64, I64, I32, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "asc_tune_save": (I32, [ctypes.c_char_p]),
    "asc_tune_load": (I32, [ctypes.c_char_p]),
    "asc_autotune_filter": (I32, [GP, P, P, I32, I64, I64, P, I64, I32, P, SZ, ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float), P]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1509_08863_amd.build` "
                               "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        # ASC_TUNE_CACHE: a tuning table saved by asc_tune_save, loaded once here
        # (the library itself reads no environment)
        cache = os.environ.get("ASC_TUNE_CACHE")
        if cache and os.path.exists(cache):
            st = L.asc_tune_load(cache.encode())
            if st != ASC_OK:
                raise AscError(st, f"ASC_TUNE_CACHE={cache}: " + L.asc_last_error().decode(errors="replace"))
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != ASC_OK:
        raise AscError(status, lib().asc_last_error().decode(errors="replace"))
