"""The C-ABI library loads and exports every symbol include/asc.h declares,
and rejects bad arguments before any launch (host logic, no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1509_08863_amd import _abi

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "asc.h")


def _declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(asc_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported_and_bound():
    L = _abi.lib()
    names = _declared()
    assert len(names) >= 15
    for nm in names:
        assert hasattr(L, nm), nm
        assert nm in _abi.SIGNATURES, f"{nm} has no ctypes signature"
    assert L.asc_abi_version() == 1


def test_workspace_queries_are_host_only():
    L = _abi.lib()
    assert L.asc_filter_workspace(1000, 32, 0, 50) > 2 * 1000 * 32 * 4
    assert L.asc_moments_workspace(100000, 64, 1, 100) > 0
    assert L.asc_lmax_workspace(10, 5) > 0
    assert L.asc_kmeans_update_workspace(1000, 8, 3) >= 1000 // 256 * 3 * 8 * 8


def _g(n=10, nnz=0, strength=True):
    fake = ctypes.c_void_p(0x1000)
    return _abi.asc_graph(n, nnz, fake, fake, None, fake if strength else None)


@pytest.mark.parametrize("case", ["p<0", "r=0", "ld<r", "ld%4", "misaligned", "no_strength", "null_Y", "ws_small"])
def test_filter_rejects_before_launch(case):
    L = _abi.lib()
    fake = ctypes.c_void_p(0x10000)
    g = _g(strength=case != "no_strength")
    p, r, ldr, ldy, R, Y, wsb = 5, 8, 8, 8, fake, fake, 1 << 30
    if case == "p<0":
        p = -1
    elif case == "r=0":
        r = 0
    elif case == "ld<r":
        ldr = 4
    elif case == "ld%4":
        ldr = 10
    elif case == "misaligned":
        R = ctypes.c_void_p(0x10004)
    elif case == "null_Y":
        Y = None
    elif case == "ws_small":
        wsb = 16
    st = L.asc_cheb_filter(ctypes.byref(g), fake, fake, p, R, 0, r, ldr, Y, ldy, None, 0, ctypes.c_void_p(0x100000),
                           wsb, None)
    assert st in (_abi.ASC_ERR_INVALID, _abi.ASC_ERR_WORKSPACE)
    assert len(L.asc_last_error()) > 0


def test_other_entry_points_reject():
    L = _abi.lib()
    fake = ctypes.c_void_p(0x10000)
    assert L.asc_cheb_coeffs(fake, 0, fake, 3, 1, fake, None) == _abi.ASC_ERR_INVALID
    assert L.asc_lmax_estimate(ctypes.byref(_g()), fake, 0, fake, None, fake, 1 << 30, None) == _abi.ASC_ERR_INVALID
    assert L.asc_kmeans_assign(fake, 10, 8, 8, fake, 0, fake, None, None) == _abi.ASC_ERR_INVALID
    assert L.asc_eigcount_dichotomy(fake, 5, fake, 3, 500, 1, fake, None, None) == _abi.ASC_ERR_INVALID
    assert L.asc_normalize_features(None, 10, 8, 8, None, None) == _abi.ASC_ERR_INVALID
    g = _abi.asc_graph(0, 0, fake, fake, None, fake)
    assert L.asc_graph_prepare(ctypes.byref(g), fake, 0, None, 0, None) == _abi.ASC_ERR_INVALID


@pytest.mark.parametrize("case", ["J=1", "k_max>128", "k_min=0", "eta>eta_max", "eta=0", "p=0", "reps=0",
                                  "null_gamma", "null_rows", "ws_small", "cols>65536"])
def test_stability_rejects_before_launch(case):
    L = _abi.lib()
    fake = ctypes.c_void_p(0x10000)
    g = _g(n=500)
    k_min, k_max, J, reps, p, steps, iters, eta_max = 2, 6, 4, 2, 20, 8, 5, 12
    etas = [2 * k for k in range(k_min, k_max + 1)]
    gamma, rows, wsb = fake, fake, 1 << 40
    if case == "J=1":
        J = 1
    elif case == "k_max>128":
        k_max, etas = 129, [4] * 128
    elif case == "k_min=0":
        k_min, etas = 0, [4] * 7
    elif case == "eta>eta_max":
        etas[-1] = eta_max + 1
    elif case == "eta=0":
        etas[0] = 0
    elif case == "p=0":
        p = 0
    elif case == "reps=0":
        reps = 0
    elif case == "null_gamma":
        gamma = None
    elif case == "null_rows":
        rows = None
    elif case == "ws_small":
        wsb = 1024
    elif case == "cols>65536":
        eta_max, J = 40000, 2
    arr = (ctypes.c_int * len(etas))(*etas)
    st = L.asc_stability(g, fake, k_min, k_max, arr, J, reps, p, steps, iters, fake, 0, eta_max, J * eta_max, rows,
                         gamma, None, None, None, None, None, fake, wsb, None)
    assert st == (_abi.ASC_ERR_WORKSPACE if case == "ws_small" else _abi.ASC_ERR_INVALID), case
    assert L.asc_last_error()


def test_stability_workspace_query():
    L = _abi.lib()
    g = _g(n=5000, nnz=50000)
    etas = [2 * k for k in range(2, 21)]
    arr = (ctypes.c_int * len(etas))(*etas)
    need = L.asc_stability_workspace(g, 2, 20, arr, 20, 20, 150, 12, 0, 40)
    # at least the state store of 151 states x 5000 rows x 800 float32 columns
    assert need >= 151 * 5000 * 800 * 4
    assert L.asc_stability_workspace(g, 2, 20, arr, 1, 20, 150, 12, 0, 40) == 0


@pytest.mark.parametrize("case", ["J=1", "k=0", "k>128", "ldl<n", "null_ari", "ws_small"])
def test_ari_rejects_before_launch(case):
    L = _abi.lib()
    fake = ctypes.c_void_p(0x10000)
    n, ldl, J, k, ari, wsb = 100, 100, 3, 4, fake, 1 << 20
    if case == "J=1":
        J = 1
    elif case == "k=0":
        k = 0
    elif case == "k>128":
        k = 129
    elif case == "ldl<n":
        ldl = 50
    elif case == "null_ari":
        ari = None
    elif case == "ws_small":
        wsb = 0
    st = L.asc_ari_pairs(fake, n, ldl, J, k, ari, None, fake, wsb, None)
    assert st == (_abi.ASC_ERR_WORKSPACE if case == "ws_small" else _abi.ASC_ERR_INVALID), case


def test_batch_plan_and_tuner_workspace_are_host_only():
    # a plan over 3 graphs of a fake 1000-node graph: planning, workspace
    # queries and argument rejection touch no device memory
    L = _abi.lib()
    fake = ctypes.c_void_p(0x1000)
    g = _g(1000, 5000)
    off = np.array([0, 100, 600, 1000], dtype=np.int64)
    ks = np.array([3, 5, 2], dtype=np.int32)
    h = ctypes.c_void_p(None)
    assert L.asc_batch_create(ctypes.byref(g), 3, off.ctypes.data, ks.ctypes.data, 48, 0, 40, 8, 0,
                              ctypes.byref(h)) == _abi.ASC_OK
    try:
        ws = L.asc_batch_workspace(h)
        tws = L.asc_batch_tune_workspace(h)
        assert ws > 2 * 1000 * 8 * 4 and tws >= ws
        # the widest candidate panel (64 float32 columns, two panels) fits
        assert tws >= 2 * 1000 * 64 * 4
        a, b, c = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_float(0.0)
        for runs, wsb, err in [(0, tws, _abi.ASC_ERR_INVALID), (101, tws, _abi.ASC_ERR_INVALID),
                               (1, tws - 1, _abi.ASC_ERR_WORKSPACE)]:
            st = L.asc_batch_autotune(h, fake, fake, 48, fake, 48, fake, None, runs, fake, wsb, ctypes.byref(a),
                                      ctypes.byref(b), ctypes.byref(c), None)
            assert st == err, (runs, wsb)
        assert L.asc_batch_autotune(None, fake, fake, 48, fake, 48, fake, None, 1, fake, tws, None, None, None,
                                    None) == _abi.ASC_ERR_INVALID
        assert L.asc_batch_workspace(h) == ws  # rejected calls leave the plan alone
    finally:
        assert L.asc_batch_destroy(h) == _abi.ASC_OK


def test_gather_probe_rejects_before_launch():
    L = _abi.lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.asc_gather_probe(None, 10, fake, 5, fake, None) == _abi.ASC_ERR_INVALID
    assert L.asc_gather_probe(fake, 0, fake, 5, fake, None) == _abi.ASC_ERR_INVALID
    assert L.asc_gather_probe(ctypes.c_void_p(0x1004), 10, fake, 5, fake, None) == _abi.ASC_ERR_INVALID
    assert L.asc_gather_probe(fake, 10, fake, 0, fake, None) == _abi.ASC_OK  # nothing to read, no launch


def test_kmeanspp_rejects_before_launch():
    L = _abi.lib()
    fake = ctypes.c_void_p(0x1000)
    ws = L.asc_kmeanspp_workspace(100)
    assert ws >= 100 * 8
    assert L.asc_kmeanspp(fake, 100, 8, 8, 0, fake, fake, fake, ws, None) == _abi.ASC_ERR_INVALID
    assert L.asc_kmeanspp(fake, 100, 8, 8, 101, fake, fake, fake, ws, None) == _abi.ASC_ERR_INVALID
    assert L.asc_kmeanspp(fake, 100, 8, 8, 5, None, fake, fake, ws, None) == _abi.ASC_ERR_INVALID
    assert L.asc_kmeanspp(fake, 100, 8, 8, 5, ctypes.c_void_p(0x1004), fake, fake, ws, None) == _abi.ASC_ERR_INVALID
    assert L.asc_kmeanspp(fake, 100, 8, 4, 5, fake, fake, fake, ws, None) == _abi.ASC_ERR_INVALID
    assert L.asc_kmeanspp(fake, 100, 8, 8, 5, fake, fake, fake, ws - 1, None) == _abi.ASC_ERR_WORKSPACE


def test_kmeans_replicates_rejects_before_launch():
    L = _abi.lib()
    fake = ctypes.c_void_p(0x1000)
    n, r, k, reps = 100, 8, 5, 4
    ws = L.asc_kmeans_replicates_workspace(n, r, k, reps)
    # per run: centroids, labels, float64 distances, inertia and stamp, then the sums' partials
    assert ws >= reps * (k * r * 4 + n * 4 + n * 8 + 8 + 4) + L.asc_kmeans_update_workspace(n, r, k)
    assert L.asc_kmeans_replicates_workspace(n, r, k, 0) == 0
    assert L.asc_kmeans_replicates_workspace(n, r, 0, reps) == 0

    def call(F=fake, ldf=r, k_=k, reps_=reps, iters=10, rows=fake, labels=fake, C=fake, inertia=fake, wsb=ws):
        return L.asc_kmeans_replicates(F, n, r, ldf, k_, reps_, iters, rows, labels, C, inertia, fake, wsb, None)

    for kw in [dict(F=None), dict(ldf=r - 1), dict(k_=0), dict(k_=1025), dict(reps_=0), dict(reps_=65536),
               dict(iters=-1), dict(iters=10001), dict(rows=None), dict(labels=None),
               dict(labels=ctypes.c_void_p(0x1002)), dict(C=ctypes.c_void_p(0x1002)),
               dict(inertia=ctypes.c_void_p(0x1004))]:
        assert call(**kw) == _abi.ASC_ERR_INVALID, kw
    assert call(wsb=ws - 1) == _abi.ASC_ERR_WORKSPACE


def test_tuning_table_round_trip_and_file_format(tmp_path):
    L = _abi.lib()
    n, nnz, r = 123457, 999, 40
    rs, var = ctypes.c_int(0), ctypes.c_int(0)
    assert L.asc_tune_set(n, nnz, r, 0, 16, 5) == _abi.ASC_OK
    path = str(tmp_path / "tune.json").encode()
    try:
        assert L.asc_tune_save(path) == _abi.ASC_OK
        assert L.asc_tune_set(n, nnz, r, 0, 0, 0) == _abi.ASC_OK  # slice_cols 0 erases the entry
        assert L.asc_tune_get(n, nnz, r, 0, ctypes.byref(rs), ctypes.byref(var)) == _abi.ASC_OK
        assert (rs.value, var.value) == (32, 0)  # the default plan for 40 float32 columns
        assert L.asc_tune_load(path) == _abi.ASC_OK
        assert L.asc_tune_get(n, nnz, r, 0, ctypes.byref(rs), ctypes.byref(var)) == _abi.ASC_OK
        assert (rs.value, var.value) == (16, 5)
        # invalid settings are rejected; a file with malformed, over-long and
        # invalid lines loads only its valid entries
        assert L.asc_tune_set(n, nnz, r, 0, 12, 0) == _abi.ASC_ERR_INVALID
        assert L.asc_tune_set(n, nnz, r, 0, 16, 16) == _abi.ASC_ERR_INVALID
        assert L.asc_tune_set(n, nnz, r, 0, 0, 0) == _abi.ASC_OK
        bad = tmp_path / "bad.json"
        bad.write_text("[\n" + "x" * 5000 + "\n"
                       + '{"n": 5, "nnz": 7, "r": 40, "dtype": 0, "slice_cols": 12, "variant": 0, "ms": 1.0},\n'
                       + '{"n": 5, "nnz": 7, "r": 40, "dtype": 3, "slice_cols": 16, "variant": 0, "ms": 1.0},\n'
                       + '{"n": 123457, "nnz": 999, "r": 40, "dtype": 0, "slice_cols": 8, "variant": 2, "ms": 0.5}\n'
                       + "]\n")
        assert L.asc_tune_load(str(bad).encode()) == _abi.ASC_OK
        assert L.asc_tune_get(n, nnz, r, 0, ctypes.byref(rs), ctypes.byref(var)) == _abi.ASC_OK
        assert (rs.value, var.value) == (8, 2)
        assert L.asc_tune_get(5, 7, 40, 0, ctypes.byref(rs), ctypes.byref(var)) == _abi.ASC_OK
        assert (rs.value, var.value) == (32, 0)
        assert L.asc_tune_load(str(tmp_path / "missing.json").encode()) == _abi.ASC_ERR_INVALID
    finally:
        L.asc_tune_set(n, nnz, r, 0, 0, 0)


def test_noalloc_filter_rejects_beyond_its_scratch_before_any_device_call():
    L = _abi.lib()
    fake = ctypes.c_void_p(0x10000)
    n, r, p = 200_000, 96, 10
    assert L.asc_filter_workspace(n, r, 0, p) > (64 << 20)
    g = _g(n, 10)
    st = L.asc_cheb_filter_noalloc(ctypes.byref(g), fake, fake, p, fake, 0, r, r, ctypes.c_void_p(0x100000000),
                                   r, None, 0, None)
    assert st == _abi.ASC_ERR_WORKSPACE
    assert b"static array" in L.asc_last_error()
    g0 = _g(10, 0)
    assert L.asc_cheb_filter_noalloc(ctypes.byref(g0), fake, fake, -1, fake, 0, 8, 8, fake, 8, None, 0,
                                     None) == _abi.ASC_ERR_INVALID


def test_tune_cache_environment_is_loaded_at_first_use(tmp_path):
    # a child process with ASC_TUNE_CACHE set sees the saved entry on first use
    import subprocess
    import sys
    path = tmp_path / "tune.json"
    path.write_text('[\n{"n": 777, "nnz": 5, "r": 24, "dtype": 0, "slice_cols": 8, "variant": 3, "ms": 0.1}\n]\n')
    code = ("import ctypes; from paper_1509_08863_amd import _abi; L = _abi.lib(); "
            "a, b = ctypes.c_int(0), ctypes.c_int(0); "
            "assert L.asc_tune_get(777, 5, 24, 0, ctypes.byref(a), ctypes.byref(b)) == 0; print(a.value, b.value)")
    env = dict(os.environ, ASC_TUNE_CACHE=str(path))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=root, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.split() == ["8", "3"]
