"""Host-side library code under AddressSanitizer and UndefinedBehaviorSanitizer.

The library's host code (argument checks, workspace sizing, plan building,
the tuning table and its file format) is compiled a second time for the host
only, with ASan and UBSan (no device code: kernels are never launched on this
path), and the ABI tests run against it in a child process with the ASan
runtime preloaded.  Any sanitizer report fails the test.  CPU only."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1509_08863_amd import build  # noqa: E402


def _asan_runtime():
    clang = os.path.join(os.path.dirname(os.path.realpath(build.HIPCC)), "..", "lib", "llvm", "bin", "clang")
    for exe in (clang, "/opt/rocm/llvm/bin/clang"):
        if os.path.exists(exe):
            r = subprocess.run([exe, "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
            path = r.stdout.strip()
            if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path):
                return path
    return None


@pytest.fixture(scope="module")
def sanitized_lib():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no ASan runtime in this toolchain")
    lib = build.build_sanitized(incremental=True)
    return lib, rt


def test_abi_tests_clean_under_asan_and_ubsan(sanitized_lib):
    lib, rt = sanitized_lib
    env = dict(os.environ)
    env["ASC_LIBRARY"] = lib
    env["LD_PRELOAD"] = rt + ((" " + env["LD_PRELOAD"]) if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONMALLOC"] = "malloc"
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q", "-x",
                        "-p", "no:cacheprovider", "-m", "not gpu"], capture_output=True, text=True, env=env,
                       cwd=ROOT, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out


def test_sanitized_library_is_instrumented_and_loaded(sanitized_lib):
    lib, rt = sanitized_lib
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report_load" in syms and "__ubsan_handle" in syms
    env = dict(os.environ)
    env["ASC_LIBRARY"] = lib
    env["LD_PRELOAD"] = rt + ((" " + env["LD_PRELOAD"]) if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0"
    code = "from paper_1509_08863_amd import _abi; _abi.lib(); print(_abi.LIB_PATH)"
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == lib


def _gcc_asan_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_cpu_baseline_clean_under_asan_and_ubsan(tmp_path):
    # the plain-C float64 recurrence (the CPU baseline the bench times) built
    # with gcc's sanitizers, run on a small weighted graph with an isolated
    # node against the NumPy oracle, in a child process with libasan preloaded
    import oracle.cpu_baseline as cb
    rt = _gcc_asan_runtime()
    if rt is None:
        pytest.skip("no gcc ASan runtime")
    lib = cb.build_sanitized(str(tmp_path / "cpu_baseline_sanitize.so"))
    env = dict(os.environ)
    env["ORACLE_CPU_BASELINE_LIB"] = lib
    env["LD_PRELOAD"] = rt + ((" " + env["LD_PRELOAD"]) if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "4"
    code = """
import numpy as np, oracle, workloads as W
import oracle.cpu_baseline as cb
assert cb.LIB.endswith('cpu_baseline_sanitize.so')
g = W.random_weighted(300, 0.05, 3, isolated=1)
w = g.w.astype(np.float64)
L = oracle.laplacian_sparse(g.n, g.row_ptr, g.col_idx, w)
lm = oracle.lmax_estimate(L, oracle.strength(g.n, g.row_ptr, g.col_idx, w), W.start_vector(g.n, 5), 60)
R = W.signals_f64(g.n, 7, 4)
for p in (0, 1, 2, 25):
    a = oracle.cheb_coeffs(0.2 * lm, lm, p)
    Y = cb.cheb_filter(g.n, g.row_ptr, g.col_idx, w, lm, a, R)
    Yo = oracle.cheb_filter(L, lm, a, R)
    assert np.max(np.abs(Y - Yo)) <= 1e-12 * max(1.0, np.max(np.abs(Yo))), p
mu = cb.cheb_moments(g.n, g.row_ptr, g.col_idx, w, lm, 25, R)
mu_o = oracle.moments(L, lm, 25, R)
assert np.max(np.abs(mu - mu_o)) <= 1e-10 * abs(mu_o[0])
print('sanitized baseline ok')
"""
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT, timeout=300)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "sanitized baseline ok" in out
