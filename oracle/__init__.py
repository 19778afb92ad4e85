"""Plain CPU oracle for brute-force incoherent dedispersion (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library: the arithmetic
lives in ``dedisp_oracle.c`` (Algorithm 1 of Sclocco et al., arXiv 1601.01165,
Section 2.1, with the delay law of Section 2, Equation 1) and in the few
NumPy FP64 helpers below (signal-to-noise, the loss built on it, and the
boxcar single-pulse search that follows dedispersion in a real-time pipeline,
Section 1).

Every function cites the passage it follows; see ``dedisp_oracle.c`` for the
per-function definitions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dedisp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math", "-ffp-contract=off"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99 + OpenMP).  Returns the path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *_CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        vp = ctypes.c_void_p
        lib.oracle_delay_samples.argtypes = [i32, vp, dbl, i32, vp, vp]
        lib.oracle_delay_samples.restype = ctypes.c_int
        lib.oracle_delay_table.argtypes = [i32, vp, dbl, i32, vp, vp]
        lib.oracle_delay_table.restype = ctypes.c_int
        lib.oracle_forward_f32.argtypes = [i32, i32, i32, i32, vp, i64, vp, vp, vp, i64]
        lib.oracle_forward_f64.argtypes = [i32, i32, i32, i32, vp, i64, vp, vp, vp, vp, i64]
        lib.oracle_forward_u8.argtypes = [i32, i32, i32, i32, vp, i64, vp, vp, i64]
        lib.oracle_forward_points_f32.argtypes = [i32, vp, i64, i64, vp, vp, i64, vp, vp, vp, vp, vp]
        lib.oracle_forward_points_u8.argtypes = [i32, vp, i64, i64, vp, i64, vp, vp, vp, vp]
        lib.oracle_adjoint_gather_f32.argtypes = [i32, i32, i32, i32, i32, vp, i64, vp, vp, vp, i64]
        lib.oracle_adjoint_scatter_f32.argtypes = [i32, i32, i32, i32, i32, vp, i64, vp, vp, vp, i64, vp]
        lib.oracle_adjoint_gather_f64.argtypes = [i32, i32, i32, i32, i32, vp, i64, vp, vp, vp, i64]
        lib.oracle_grad_w.argtypes = [i32, i32, i32, i32, vp, i64, vp, i64, vp, vp, vp]
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def num_threads() -> int:
    """OpenMP threads the oracle runs on."""
    return int(_load().oracle_num_threads())


# --------------------------------------------------------------------------
# Section 2, Equation 1: delay law and its integer table.
# --------------------------------------------------------------------------

def delay_samples(freq_mhz, tsamp_s, dm) -> np.ndarray:
    """Unrounded delays x[dm][chan] = 4150*DM*(1/f^2 - 1/f_h^2)/tsamp (Eq. 1)."""
    f = _c(freq_mhz, np.float64)
    d = _c(dm, np.float64)
    x = np.empty((d.size, f.size), np.float64)
    if _load().oracle_delay_samples(f.size, _p(f), float(tsamp_s), d.size, _p(d), _p(x)) != 0:
        raise ValueError("invalid delay-law arguments")
    return x


def delay_table(freq_mhz, tsamp_s, dm) -> np.ndarray:
    """Integer delays delta[dm][chan] = floor(x + 1/2) of Eq. 1 (int32)."""
    f = _c(freq_mhz, np.float64)
    d = _c(dm, np.float64)
    t = np.empty((d.size, f.size), np.int32)
    if _load().oracle_delay_table(f.size, _p(f), float(tsamp_s), d.size, _p(d), _p(t)) != 0:
        raise ValueError("invalid delay-law arguments")
    return t


# --------------------------------------------------------------------------
# Section 2.1, Algorithm 1: forward dedispersion.
# --------------------------------------------------------------------------

def _shape_in(x):
    if x.ndim == 2:
        x = x[None]
    return x


def forward_f32(x, delta, nsamp, w=None) -> np.ndarray:
    """Algorithm 1 in FP32: out[b][dm][s] = sum_c w[c]*x[b][c][s+delta[dm][c]].

    ``x`` is [nbeam][nchan][nin] (or [nchan][nin]); returns [nbeam][ndm][nsamp].
    """
    x = _c(_shape_in(x), np.float32)
    delta = _c(delta, np.int32)
    nb, nc, nin = x.shape
    nd = delta.shape[0]
    assert delta.shape[1] == nc and nin >= nsamp + int(delta.max())
    wv = None if w is None else _c(w, np.float32)
    out = np.empty((nb, nd, nsamp), np.float32)
    _load().oracle_forward_f32(nb, nc, nd, nsamp, _p(x), nin, _p(delta), _p(wv), _p(out), nsamp)
    return out


def forward_f64(x, delta, nsamp, w=None, with_scale=False):
    """Algorithm 1 in FP64; with ``with_scale`` also returns sum_c |w*x|."""
    x = _c(_shape_in(x), np.float64)
    delta = _c(delta, np.int32)
    nb, nc, nin = x.shape
    nd = delta.shape[0]
    assert delta.shape[1] == nc and nin >= nsamp + int(delta.max())
    wv = None if w is None else _c(w, np.float64)
    out = np.empty((nb, nd, nsamp), np.float64)
    sc = np.empty_like(out) if with_scale else None
    _load().oracle_forward_f64(nb, nc, nd, nsamp, _p(x), nin, _p(delta), _p(wv), _p(out), _p(sc), nsamp)
    return (out, sc) if with_scale else out


def forward_u8(x, delta, nsamp) -> np.ndarray:
    """Algorithm 1 on uint8 input with an int32 accumulator (unit weights)."""
    x = _c(_shape_in(x), np.uint8)
    delta = _c(delta, np.int32)
    nb, nc, nin = x.shape
    nd = delta.shape[0]
    assert delta.shape[1] == nc and nin >= nsamp + int(delta.max())
    out = np.empty((nb, nd, nsamp), np.int32)
    _load().oracle_forward_u8(nb, nc, nd, nsamp, _p(x), nin, _p(delta), _p(out), nsamp)
    return out


def forward_points(x, delta, beams, dms, samples, w=None):
    """Selected outputs of Algorithm 1, one by one.

    For float32 input returns (values float32, scale float64 = sum_c |w*x|);
    for uint8 input returns (values int32, None).
    """
    x = _shape_in(x)
    assert x.flags["C_CONTIGUOUS"]
    delta = _c(delta, np.int32)
    nb, nc, nin = x.shape
    pb, pd, ps = (_c(a, np.int32) for a in (beams, dms, samples))
    n = pb.size
    assert pb.size == pd.size == ps.size
    assert n == 0 or (pb.min() >= 0 and pb.max() < nb and pd.min() >= 0 and pd.max() < delta.shape[0])
    assert n == 0 or (ps.min() >= 0 and int(ps.max()) + int(delta.max()) < nin)
    if x.dtype == np.uint8:
        out = np.empty(n, np.int32)
        _load().oracle_forward_points_u8(nc, _p(x), nin, nc * nin, _p(delta), n, _p(pb), _p(pd), _p(ps), _p(out))
        return out, None
    assert x.dtype == np.float32
    wv = None if w is None else _c(w, np.float32)
    out = np.empty(n, np.float32)
    sc = np.empty(n, np.float64)
    _load().oracle_forward_points_f32(nc, _p(x), nin, nc * nin, _p(delta), _p(wv), n, _p(pb), _p(pd), _p(ps),
                                      _p(out), _p(sc))
    return out, sc


# --------------------------------------------------------------------------
# Transpose of Algorithm 1 (adjoint) and the weight gradient.
# --------------------------------------------------------------------------

def adjoint_gather_f32(g, delta, nin, w=None) -> np.ndarray:
    """grad_in[b][c][t] = w[c] * sum_{dm asc, 0<=t-delta<nsamp} g[b][dm][t-delta[dm][c]]."""
    g = _c(_shape_in(g), np.float32)
    delta = _c(delta, np.int32)
    nb, nd, ns = g.shape
    nc = delta.shape[1]
    wv = None if w is None else _c(w, np.float32)
    out = np.empty((nb, nc, nin), np.float32)
    _load().oracle_adjoint_gather_f32(nb, nc, nd, ns, nin, _p(g), ns, _p(delta), _p(wv), _p(out), nin)
    return out


def adjoint_scatter_f32(g, delta, nin, w=None) -> np.ndarray:
    """The same transpose, computed by pushing each g element to the input it read."""
    g = _c(_shape_in(g), np.float32)
    delta = _c(delta, np.int32)
    nb, nd, ns = g.shape
    nc = delta.shape[1]
    stride = max(nin, ns + int(delta.max()))
    wv = None if w is None else _c(w, np.float32)
    out = np.empty((nb, nc, stride), np.float32)
    tmp = np.empty((nb, nc, stride), np.float32)
    _load().oracle_adjoint_scatter_f32(nb, nc, nd, ns, nin, _p(g), ns, _p(delta), _p(wv), _p(out), stride, _p(tmp))
    return np.ascontiguousarray(out[:, :, :nin])


def adjoint_gather_f64(g, delta, nin):
    """FP64 G (without the weight) and its scale sum |g| over the same terms."""
    g = _c(_shape_in(g), np.float64)
    delta = _c(delta, np.int32)
    nb, nd, ns = g.shape
    nc = delta.shape[1]
    G = np.empty((nb, nc, nin), np.float64)
    A = np.empty_like(G)
    _load().oracle_adjoint_gather_f64(nb, nc, nd, ns, nin, _p(g), ns, _p(delta), _p(G), _p(A), nin)
    return G, A


def grad_w(x, g, delta):
    """d/dw[c] of sum g*out: sum_b,dm,s g[b][dm][s]*x[b][c][s+delta[dm][c]] (FP64), and its scale."""
    x = _c(_shape_in(x), np.float32)
    g = _c(_shape_in(g), np.float32)
    delta = _c(delta, np.int32)
    nb, nc, nin = x.shape
    _, nd, ns = g.shape
    assert nin >= ns + int(delta.max())
    gw = np.empty(nc, np.float64)
    ab = np.empty(nc, np.float64)
    _load().oracle_grad_w(nb, nc, nd, ns, _p(x), nin, _p(g), ns, _p(delta), _p(gw), _p(ab))
    return gw, ab


# --------------------------------------------------------------------------
# Signal-to-noise of a dedispersed series and the loss built on it.  Not in
# the paper's method (it mentions S/N only in passing); used as the training
# objective of the differentiable workload.  FP64, NumPy.
# --------------------------------------------------------------------------

def snr(y) -> float:
    """(max - mean) / std of one series (population std, ddof = 0)."""
    y = np.asarray(y, np.float64)
    return float((y.max() - y.mean()) / y.std())


def snr_loss(out, picks) -> float:
    """Negative mean S/N over the (beam, dm) rows in ``picks``."""
    return -float(np.mean([snr(out[b, j]) for b, j in picks]))


def snr_grad(y) -> np.ndarray:
    """Gradient of snr(y) with respect to y (argmax ties go to the lowest index)."""
    y = np.asarray(y, np.float64)
    n = y.size
    m = y.mean()
    sd = y.std()
    k = int(np.argmax(y))
    num = y[k] - m
    dnum = np.full(n, -1.0 / n)
    dnum[k] += 1.0
    dsd = (y - m) / (n * sd)
    return dnum / sd - num * dsd / (sd * sd)


# --------------------------------------------------------------------------
# Single-pulse search over dedispersed series (the real-time detection that
# dedispersion feeds, Section 1; the paper does not define it, so the search
# here is the textbook boxcar matched filter).  FP64, NumPy, one row at a time.
#
#   widths      w_k = 2^k for k < nwidth, skipping widths longer than the row
#   B_w(t)      sum of y[t .. t + w) for 0 <= t <= n - w
#   mean, std   of the whole row (population std, ddof = 0)
#   S/N_w       (max_t B_w(t) - w * mean) / (std * sqrt(w)); 0 when std == 0
#   result      the width with the largest S/N (ties: the narrower), the first
#               t reaching that width's maximum, its S/N, mean and std
# --------------------------------------------------------------------------

def boxcar_sums(y, w) -> np.ndarray:
    """B_w(t) for every full window of the row, each summed directly in FP64."""
    y = np.asarray(y, np.float64)
    return np.lib.stride_tricks.sliding_window_view(y, w).sum(axis=1)


def detect_row(y, nwidth):
    """(snr, width, start, mean, std) of one dedispersed series."""
    y = np.asarray(y, np.float64)
    n = y.size
    mean = float(y.mean())
    std = float(y.std())
    best = None
    for k in range(nwidth):
        w = 1 << k
        if w > n:
            break
        b = boxcar_sums(y, w)
        t = int(np.argmax(b))
        s = (float(b[t]) - w * mean) / (std * np.sqrt(w)) if std > 0 else 0.0
        if best is None or s > best[0]:
            best = (s, w, t)
    return best[0], best[1], best[2], mean, std


def detect(rows, nwidth):
    """Search every row of rows [..., nsamp]; returns a dict of arrays of the
    leading shape: snr (f8), width (i4), start (i4), mean (f8), std (f8)."""
    rows = np.asarray(rows)
    lead = rows.shape[:-1]
    flat = rows.reshape(-1, rows.shape[-1])
    res = [detect_row(r, nwidth) for r in flat]
    out = {}
    for i, (name, dt) in enumerate((("snr", np.float64), ("width", np.int32), ("start", np.int32),
                                    ("mean", np.float64), ("std", np.float64))):
        out[name] = np.array([r[i] for r in res], dt).reshape(lead)
    return out

