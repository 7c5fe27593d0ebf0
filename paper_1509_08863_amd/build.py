"""Builds libasc.so (the HIP library behind include/asc.h) for gfx950, in-tree.

    python -m paper_1509_08863_amd.build [--incremental | --sanitize]

Every .hip under csrc/ is compiled with hipcc into _build/*.o and linked into
paper_1509_08863_amd/libasc.so.  Packed-FP32 instruction selection is turned
off for all device code.  With --incremental only sources newer than their
object are recompiled (all of them if a header is newer than the oldest
object); the default always recompiles everything.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libasc.so")
ARCH = os.environ.get("ASC_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

CFLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
    cmd = [HIPCC, *CFLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def _obj_of(src: str) -> str:
    return os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))


def _stale(srcs):
    objs = [_obj_of(s) for s in srcs]
    if not all(os.path.exists(o) for o in objs):
        return [s for s, o in zip(srcs, objs) if not os.path.exists(o)] or srcs
    oldest = min(os.path.getmtime(o) for o in objs)
    headers = glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    if any(os.path.getmtime(h) > oldest for h in headers):
        return srcs
    return [s for s, o in zip(srcs, objs) if os.path.getmtime(s) > os.path.getmtime(o)]


def build(verbose: bool = False, incremental: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    todo = _stale(srcs) if incremental else srcs
    if todo:
        with cf.ThreadPoolExecutor(max_workers=min(8, len(todo))) as ex:
            list(ex.map(_compile, todo))
    objs = [_obj_of(s) for s in srcs]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


# Host-only build for the sanitizers: every source compiled for the host alone
# (relocatable device code with no device part, so nothing is compiled for the
# GPU and no kernel can run), with AddressSanitizer and UndefinedBehaviorSanitizer
# on the host code, linked into _build/sanitize/libasc_sanitize.so.  Loading it
# needs the ASan runtime preloaded; it serves the argument checks, workspace
# sizing, planning and tuning-table code of the CPU tests.
SANITIZE_DIR = os.path.join(BUILD, "sanitize")
SANITIZE_LIB = os.path.join(SANITIZE_DIR, "libasc_sanitize.so")
SANITIZE_FLAGS = [
    f"--offload-arch={ARCH}", "-fgpu-rdc", "--offload-host-only",
    "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]


def _compile_sanitized(src: str) -> str:
    obj = os.path.join(SANITIZE_DIR, os.path.basename(src).replace(".hip", ".o"))
    r = subprocess.run([HIPCC, *SANITIZE_FLAGS, "-c", src, "-o", obj], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc (sanitize) failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build_sanitized(verbose: bool = False, incremental: bool = False) -> str:
    os.makedirs(SANITIZE_DIR, exist_ok=True)
    srcs = sources()
    deps = srcs + glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    if incremental and os.path.exists(SANITIZE_LIB) and \
            os.path.getmtime(SANITIZE_LIB) >= max(os.path.getmtime(d) for d in deps):
        return SANITIZE_LIB
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile_sanitized, srcs))
    tmp = SANITIZE_LIB + ".tmp"
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-fgpu-rdc", "--hip-link", "-shared", "-fPIC", *objs,
                        "-o", tmp], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link (sanitize) failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, SANITIZE_LIB)
    if verbose:
        print("built", SANITIZE_LIB)
    return SANITIZE_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv[1:]:
        build_sanitized(verbose=True)
    else:
        build(verbose=True, incremental="--incremental" in sys.argv[1:])
    sys.exit(0)
