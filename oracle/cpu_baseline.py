"""ctypes loader of the plain-C FP64 CPU baseline (cpu_baseline.c).  Test
infrastructure only; built by ``build()`` (gcc -O2 -fopenmp)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_baseline.c")
# ORACLE_CPU_BASELINE_LIB names another build of the same source (the
# sanitizer build of the host checks); by default the in-tree library
LIB = os.environ.get("ORACLE_CPU_BASELINE_LIB") or os.path.join(HERE, "_cpu_baseline.so")


def build_sanitized(out_path: str) -> str:
    """The same source under AddressSanitizer and UndefinedBehaviorSanitizer
    (gcc), for the host sanitizer test; loading it needs libasan preloaded."""
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared", "-std=c99", SRC, "-o", out_path]
    subprocess.check_call(cmd)
    return out_path


def build() -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", SRC, "-o", LIB + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built() -> str:
    """Builds the library if it is missing or older than its source."""
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        return build()
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError("oracle CPU baseline not built: call oracle.cpu_baseline.build()")
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        lib.oracle_cheb_filter.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_double, P, ctypes.c_int,
                                           P, ctypes.c_int64, P]
        lib.oracle_cheb_filter.restype = ctypes.c_int
        lib.oracle_cheb_moments.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_double, ctypes.c_int, P,
                                            ctypes.c_int64, P]
        lib.oracle_cheb_moments.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_threads(t: int) -> None:
    _load().oracle_set_threads(int(t))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cheb_filter(n, row_ptr, col_idx, w, lmax, a, R):
    """Y = sum_j a_j T_j(L~) R in float64 (w None for unit weights)."""
    lib = _load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    w64 = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    Y = np.empty_like(R)
    rc = lib.oracle_cheb_filter(n, rp.ctypes.data, ci.ctypes.data, None if w64 is None else w64.ctypes.data,
                                float(lmax), a.ctypes.data, len(a) - 1, R.ctypes.data, R.shape[1], Y.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle CPU baseline allocation failed")
    return Y


def cheb_moments(n, row_ptr, col_idx, w, lmax, p, R):
    """mu_j = <R, T_j(L~) R>_F, j = 0..p, in float64 (w None for unit weights)."""
    lib = _load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    w64 = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    mu = np.empty(p + 1, dtype=np.float64)
    rc = lib.oracle_cheb_moments(n, rp.ctypes.data, ci.ctypes.data, None if w64 is None else w64.ctypes.data,
                                 float(lmax), int(p), R.ctypes.data, R.shape[1], mu.ctypes.data)
    if rc != 0:
        raise MemoryError("oracle CPU baseline allocation failed")
    return mu
