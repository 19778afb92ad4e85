"""Build libdedisp.so (gfx950) in-tree with hipcc.

Usage: python -m paper_1601_01165_amd.build [--incremental]

By default every source is compiled.  --incremental recompiles only the
objects older than their source or any shared header (a development aid).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libdedisp.so")
BUILD_DIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed FP32 instructions are switched off for all device code; every
# source is compiled with FP contraction off so that only explicit fmaf()
# calls fuse.
DEVICE_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE,
    "-Wall", "-Wno-unused-function",
]

SOURCES = ["engine.hip", "detect.hip", "plan.cpp", "batch.cpp", "tune.cpp", "detect.cpp"]


def _gen():
    subprocess.run([sys.executable, os.path.join(CSRC, "gen_win_asm.py"), os.path.join(CSRC, "win_asm.inc")],
                   check=True)


def _stale(src: str, obj: str) -> bool:
    if not os.path.exists(obj):
        return True
    deps = [os.path.join(CSRC, src), os.path.join(INCLUDE, "dedisp.h")]
    deps += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".h", ".inc"))]
    return os.path.getmtime(obj) < max(os.path.getmtime(d) for d in deps)


def _compile(src: str, force: bool = True) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    if not force and not _stale(src, obj):
        return obj
    cmd = [HIPCC, *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *DEVICE_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stdout}\n{r.stderr}")
    return obj


def build(force: bool = True) -> str:
    """Compile every source for gfx950 and link libdedisp.so.  Returns its path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    _gen()
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(lambda f: _compile(f, force), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def device_asm(src: str = "engine.hip") -> str:
    """Device assembly of one source (for inspection of register use)."""
    out = os.path.join(BUILD_DIR, os.path.basename(src) + ".s")
    os.makedirs(BUILD_DIR, exist_ok=True)
    cmd = [HIPCC, *DEVICE_FLAGS, "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


if __name__ == "__main__":
    print(build(force="--incremental" not in sys.argv[1:]))
