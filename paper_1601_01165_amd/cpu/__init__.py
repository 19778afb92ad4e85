"""Tuned multi-core CPU dedispersion: the paper's CPU comparison (Section 5)
built with OpenMP and SIMD, behind the C-ABI of include/dedisp_cpu.h.

Host arrays only (NumPy).  ``autotune`` times every tile configuration on the
given data and returns the fastest, as the paper tunes its CPU code too.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dedisp_cpu.cpp")
LIB = os.path.join(HERE, "libdedisp_cpu.so")
_BUILD = os.path.join(HERE, "_build")

_COMMON = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-ffp-contract=off", "-fno-math-errno"]
_ISAS = [("ddcpu_avx512", ["-mavx512f", "-mavx512bw", "-mfma", "-mprefer-vector-width=512"]),
         ("ddcpu_avx2", ["-mavx2", "-mfma"]),
         ("ddcpu_generic", [])]


def build() -> str:
    """Compile one kernel copy per instruction set plus the dispatcher; link libdedisp_cpu.so."""
    os.makedirs(_BUILD, exist_ok=True)

    def one(job):
        name, flags = job
        obj = os.path.join(_BUILD, name + ".o")
        subprocess.run(["g++", *_COMMON, *flags, f"-DDDCPU_NS={name}", "-c", SRC, "-o", obj], check=True)
        return obj

    jobs = _ISAS + [("ddcpu_dispatch", ["-DDDCPU_DISPATCH"])]
    with ThreadPoolExecutor(4) as ex:
        objs = list(ex.map(one, jobs))
    tmp = LIB + ".tmp"
    subprocess.run(["g++", "-shared", "-fopenmp", *objs, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


def build_if_missing() -> str:
    return LIB if os.path.exists(LIB) else build()


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: build it with paper_1601_01165_amd.cpu.build()")
        L = ctypes.CDLL(LIB)
        i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        L.ddcpu_forward_f32.argtypes = [i32, i32, i32, i32, vp, i64, vp, vp, vp, i64, i32]
        L.ddcpu_forward_f32.restype = ctypes.c_int
        L.ddcpu_forward_u8.argtypes = [i32, i32, i32, i32, vp, i64, vp, vp, i64, i32]
        L.ddcpu_forward_u8.restype = ctypes.c_int
        L.ddcpu_num_configs.restype = i32
        L.ddcpu_config.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.ddcpu_config.restype = ctypes.c_int
        L.ddcpu_num_threads.restype = i32
        L.ddcpu_isa.restype = ctypes.c_char_p
        _lib = L
    return _lib


def configs():
    """[(dt, tt), ...] in configuration order."""
    L = lib()
    out = []
    for i in range(L.ddcpu_num_configs()):
        dt, tt = ctypes.c_int32(), ctypes.c_int32()
        L.ddcpu_config(i, ctypes.byref(dt), ctypes.byref(tt))
        out.append((dt.value, tt.value))
    return out


def num_threads() -> int:
    return int(lib().ddcpu_num_threads())


def isa() -> str:
    return lib().ddcpu_isa().decode()


def forward(x: np.ndarray, delta: np.ndarray, nsamp: int, w: np.ndarray | None = None, cfg: int = 3,
            out: np.ndarray | None = None) -> np.ndarray:
    """x [nbeam][nchan][nin] (float32 or uint8), delta [ndm][nchan] int32 -> out [nbeam][ndm][nsamp]."""
    x3 = x if x.ndim == 3 else x[None]
    if x3.strides[2] != x3.itemsize or x3.strides[0] != x3.shape[1] * x3.strides[1]:
        x3 = np.ascontiguousarray(x3)
    nb, nc, nin = x3.shape
    d = np.ascontiguousarray(delta, dtype=np.int32)
    nd = d.shape[0]
    if d.shape[1] != nc:
        raise ValueError("delta must be [ndm][nchan]")
    u8 = x3.dtype == np.uint8
    if not u8 and x3.dtype != np.float32:
        raise ValueError("input must be float32 or uint8")
    if out is None:
        out = np.empty((nb, nd, nsamp), np.int32 if u8 else np.float32)
    is_ = x3.strides[1] // x3.itemsize
    os_ = out.strides[1] // out.itemsize
    L = lib()
    if u8:
        if w is not None:
            raise ValueError("weights are not supported for uint8 input")
        st = L.ddcpu_forward_u8(nb, nc, nd, nsamp, x3.ctypes.data, is_, d.ctypes.data, out.ctypes.data, os_, cfg)
    else:
        wp = None
        if w is not None:
            w = np.ascontiguousarray(w, dtype=np.float32)
            wp = w.ctypes.data
        st = L.ddcpu_forward_f32(nb, nc, nd, nsamp, x3.ctypes.data, is_, d.ctypes.data, wp, out.ctypes.data, os_,
                                 cfg)
    if st != 0:
        raise ValueError("ddcpu_forward rejected the arguments")
    return out if x.ndim == 3 else out[0]


def autotune(x: np.ndarray, delta: np.ndarray, nsamp: int, w: np.ndarray | None = None, reps: int = 1):
    """Time every configuration (best of `reps` after one warm-up) -> ({(dt, tt): seconds}, best cfg index)."""
    out = None
    times = {}
    best, best_t = 0, float("inf")
    for i, c in enumerate(configs()):
        out = forward(x, delta, nsamp, w, i, out)
        t = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            forward(x, delta, nsamp, w, i, out)
            t = min(t, time.perf_counter() - t0)
        times[c] = t
        if t < best_t:
            best, best_t = i, t
    return times, best
