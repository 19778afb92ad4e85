"""Brute-force incoherent dedispersion on MI355X (gfx950).

Thin Python binding of libdedisp.so (see include/dedisp.h): argument
marshalling only, every step of the computation runs in the library's HIP
kernels.  PyTorch supplies device memory and streams.

Method: Sclocco et al., "Real-Time Dedispersion for Fast Radio Transient
Surveys, using Auto Tuning on Many-Core Accelerators" (arXiv 1601.01165):
delays from Section 2, Equation 1; the sum of Section 2.1, Algorithm 1.

Tensors
  input   [nbeam][nchan][nin]   float32 or uint8 on the GPU, time contiguous
  output  [nbeam][ndm][nsamp]   float32 (int32 for uint8 input)
Each row's byte stride must be a multiple of 16 and the base pointer 16-byte
aligned; ``empty_rows`` allocates such tensors (a padded buffer, returned as a
view), and inputs that do not satisfy this are copied into one.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _clib
from ._clib import F32, I32, U8, DedispError, check

__all__ = [
    "Plan", "Batch", "DedispFunction", "DedispError", "compute_delays", "dedisperse", "dedisperse_autograd",
    "adjoint", "adjoint_noalloc", "empty_rows", "variant_names", "lib", "detect", "detect_rows",
]


def lib():
    return _clib.load()


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dt(dtype) -> int:
    if dtype in (torch.float32, np.float32, "f32", "float32", F32):
        return F32
    if dtype in (torch.uint8, np.uint8, "u8", "uint8", U8):
        return U8
    raise ValueError(f"unsupported dtype {dtype}")


def _esz(dtype: torch.dtype) -> int:
    return torch.empty((), dtype=dtype).element_size()


def padded(n: int, elem_bytes: int) -> int:
    """Smallest row length >= n whose byte size is a multiple of 16."""
    q = 16 // elem_bytes
    return (n + q - 1) // q * q


def empty_rows(nbeam: int, nrows: int, n: int, dtype=torch.float32, device="cuda", zero=False) -> torch.Tensor:
    """A [nbeam][nrows][n] tensor whose rows start on 16-byte boundaries."""
    stride = padded(n, _esz(dtype))
    buf = (torch.zeros if zero else torch.empty)((nbeam, nrows, stride), dtype=dtype, device=device)
    return buf[:, :, :n]


def _rows_ok(t: torch.Tensor) -> bool:
    es = t.element_size()
    return (t.dim() == 3 and t.stride(2) == 1 and (t.stride(1) * es) % 16 == 0
            and t.stride(0) == t.shape[1] * t.stride(1) and t.data_ptr() % 16 == 0)


def _as_rows(t: torch.Tensor) -> torch.Tensor:
    """t as [nbeam][rows][n] satisfying the row rules (copying if needed)."""
    if t.dim() == 2:
        t = t.unsqueeze(0)
    if t.dim() != 3:
        raise ValueError("expected a [nbeam][rows][samples] or [rows][samples] tensor")
    if not t.is_cuda:
        raise ValueError("tensors must be on the GPU")
    if _rows_ok(t):
        return t
    r = empty_rows(t.shape[0], t.shape[1], t.shape[2], t.dtype, t.device)
    r.copy_(t)
    return r


def variant_names(dtype="f32") -> list[str]:
    L = lib()
    d = _dt(dtype)
    return [L.dedisp_variant_name(d, i).decode() for i in range(L.dedisp_variant_count(d))]


def compute_delays(freq_mhz, tsamp_s: float, dms) -> np.ndarray:
    """Host-only delay table delta[dm][chan] (Eq. 1, FP64, round half up)."""
    f = np.ascontiguousarray(freq_mhz, np.float64)
    d = np.ascontiguousarray(dms, np.float64)
    out = np.empty((d.size, f.size), np.int32)
    md = ctypes.c_int32()
    check(lib().dedisp_compute_delays(f.size, f.ctypes.data, float(tsamp_s), d.size, d.ctypes.data,
                                      out.ctypes.data, ctypes.byref(md)), "compute_delays")
    return out


class Plan:
    """Delay table for one observing set-up and DM list, resident on the GPU."""

    def __init__(self, freq_mhz, tsamp_s: float, dms):
        L = lib()
        f = np.ascontiguousarray(freq_mhz, np.float64)
        d = np.ascontiguousarray(dms, np.float64)
        h = ctypes.c_void_p()
        check(L.dedisp_plan_create(ctypes.byref(h), f.size, f.ctypes.data, float(tsamp_s), d.size, d.ctypes.data),
              "plan_create")
        self._h = h
        nc, nd, md = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(L.dedisp_plan_info(h, ctypes.byref(nc), ctypes.byref(nd), ctypes.byref(md)), "plan_info")
        self.nchan, self.ndm, self.max_delay = nc.value, nd.value, md.value
        self.freq_mhz, self.tsamp_s, self.dms = f.copy(), float(tsamp_s), d.copy()

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dedisp_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def delays(self) -> np.ndarray:
        out = np.empty((self.ndm, self.nchan), np.int32)
        check(lib().dedisp_plan_delays(self._h, out.ctypes.data), "plan_delays")
        return out

    def prepare(self, dtype="f32", adjoint=False):
        check(lib().dedisp_plan_prepare(self._h, _dt(dtype), int(bool(adjoint))), "plan_prepare")

    def set_variant(self, index: int, dtype="f32"):
        check(lib().dedisp_plan_set_variant(self._h, _dt(dtype), int(index)), "plan_set_variant")

    def variant(self, dtype="f32") -> int:
        return int(lib().dedisp_plan_variant(self._h, _dt(dtype)))

    def set_adjoint_variant(self, index: int):
        check(lib().dedisp_plan_set_adjoint_variant(self._h, int(index)), "plan_set_adjoint_variant")

    def adjoint_variant(self) -> int:
        return int(lib().dedisp_plan_adjoint_variant(self._h))

    def detect_variant(self, dtype="f32") -> int:
        """Variant with the single-pulse search in its epilogue that detect
        uses for dtype (-1: the unfused path)."""
        return int(lib().dedisp_detect_variant(self.handle, _dt(dtype)))

    def autotune_adjoint(self, nbeam: int, nsamp: int) -> dict:
        """Time every adjoint variant and the direct adjoint, keep the
        fastest; returns {variant name or "direct": ms}."""
        names = variant_names("f32")
        ms = (ctypes.c_float * (len(names) + 1))()
        check(lib().dedisp_autotune_adjoint(self.handle, nbeam, nsamp, ms, len(names) + 1), "autotune_adjoint")
        out = {n: float(ms[i]) for i, n in enumerate(names) if ms[i] > 0}
        if ms[len(names)] > 0:
            out["direct"] = float(ms[len(names)])
        return out

    def set_detect_variant(self, index: int, dtype="f32"):
        """Force the search path: a fused variant, -1 unfused, -2 automatic."""
        check(lib().dedisp_plan_set_detect_variant(self.handle, _dt(dtype), index), "set_detect_variant")

    def autotune_detect(self, nbeam: int, nsamp: int, dtype="f32", nwidth: int = 6) -> dict:
        """Time the fused variants and the unfused path of the single-pulse
        search, keep the fastest; returns {variant name or "unfused": ms}."""
        names = variant_names(dtype)
        ms = (ctypes.c_float * (len(names) + 1))()
        check(lib().dedisp_detect_autotune(self.handle, nbeam, nsamp, _dt(dtype), nwidth, ms, len(names) + 1),
              "detect_autotune")
        out = {n: float(ms[i]) for i, n in enumerate(names) if ms[i] > 0}
        if ms[len(names)] > 0:
            out["unfused"] = float(ms[len(names)])
        return out

    def autotune(self, nbeam: int, nsamp: int, dtype="f32", cache_path: str | None = None) -> dict:
        """Exhaustive search over the compiled variants; returns {name: ms}."""
        L = lib()
        d = _dt(dtype)
        check(L.dedisp_autotune(self._h, int(nbeam), int(nsamp), d, cache_path.encode() if cache_path else None),
              "autotune")
        n = L.dedisp_variant_count(d) + 1
        ms = np.full(n, -1.0, np.float32)
        k = L.dedisp_autotune_times(self._h, d, ms.ctypes.data, n)
        names = variant_names(dtype) + ["direct"]
        return {names[i]: float(ms[i]) for i in range(k)}


def dedisperse(x: torch.Tensor, plan: Plan, w: torch.Tensor | None = None, nsamp: int | None = None,
               out: torch.Tensor | None = None) -> torch.Tensor:
    """out[b][dm][t] = sum_c w[c] * x[b][c][t + delta[dm][c]] (Algorithm 1)."""
    squeeze = x.dim() == 2
    xr = _as_rows(x)
    nb, nc, nin = xr.shape
    if nc != plan.nchan:
        raise ValueError(f"input has {nc} channels, plan has {plan.nchan}")
    if nsamp is None:
        nsamp = nin - plan.max_delay
    if nsamp < 1 or nin < nsamp + plan.max_delay:
        raise ValueError(f"need nin >= nsamp + max_delay ({nsamp} + {plan.max_delay}), got {nin}")
    dt = _dt(xr.dtype)
    odt = torch.int32 if dt == U8 else torch.float32
    if w is not None:
        if dt == U8:
            raise ValueError("weights are not supported for uint8 input")
        w = w.detach().to(torch.float32).contiguous()
        if w.numel() != nc or not w.is_cuda:
            raise ValueError("weights must be a float32 GPU tensor of nchan values")
    if out is None:
        out = empty_rows(nb, plan.ndm, nsamp, odt, xr.device)
    elif not _rows_ok(out) or out.dtype != odt or tuple(out.shape) != (nb, plan.ndm, nsamp):
        raise ValueError("out must be [nbeam][ndm][nsamp] with 16-byte aligned rows")
    check(lib().dedisp_execute(plan.handle, nb, nsamp, ctypes.c_void_p(xr.data_ptr()), dt, xr.stride(1),
                               ctypes.c_void_p(w.data_ptr()) if w is not None else None,
                               ctypes.c_void_p(out.data_ptr()), I32 if dt == U8 else F32, out.stride(1),
                               _stream(xr.device)), "execute")
    return out[0] if squeeze else out


def adjoint(g: torch.Tensor, plan: Plan, nin: int, w: torch.Tensor | None = None, x: torch.Tensor | None = None,
            want_grad_in: bool = True):
    """Transpose of dedisperse.  Returns (grad_in [nbeam][nchan][nin] or None,
    grad_w [nchan] or None); grad_w needs the forward input x."""
    gr = _as_rows(g.to(torch.float32) if g.dtype != torch.float32 else g)
    nb, nd, ns = gr.shape
    if nd != plan.ndm:
        raise ValueError(f"gradient has {nd} DM rows, plan has {plan.ndm}")
    if w is not None:
        w = w.detach().to(torch.float32).contiguous()
    xr = _as_rows(x.detach()) if x is not None else None
    gi = empty_rows(nb, plan.nchan, nin, torch.float32, gr.device) if want_grad_in else None
    gw = torch.empty(plan.nchan, dtype=torch.float32, device=gr.device) if xr is not None else None
    ws = None
    nbytes = 0
    if gw is not None:
        nbytes = lib().dedisp_adjoint_workspace_bytes(plan.handle, nb, nin)
        ws = torch.empty(max(nbytes, 8), dtype=torch.uint8, device=gr.device)
    check(lib().dedisp_adjoint(plan.handle, nb, ns, nin, ctypes.c_void_p(gr.data_ptr()), gr.stride(1),
                               ctypes.c_void_p(w.data_ptr()) if w is not None else None,
                               ctypes.c_void_p(xr.data_ptr()) if xr is not None else None,
                               xr.stride(1) if xr is not None else 0,
                               ctypes.c_void_p(gi.data_ptr()) if gi is not None else None,
                               gi.stride(1) if gi is not None else 0,
                               ctypes.c_void_p(gw.data_ptr()) if gw is not None else None,
                               ctypes.c_void_p(ws.data_ptr()) if ws is not None else None, nbytes,
                               _stream(gr.device)), "adjoint")
    return gi, gw


def adjoint_noalloc(g: torch.Tensor, plan: Plan, nin: int, w: torch.Tensor | None = None,
                    x: torch.Tensor | None = None, grad_in: torch.Tensor | None = None,
                    grad_w: torch.Tensor | None = None):
    """adjoint() through the allocation-free entry point: the caller passes
    the outputs (grad_in [nbeam][nchan][nin] with 16-byte rows, grad_w [nchan]
    float32, either may be None) and nothing is allocated, by this function or
    the library; the plan's adjoint kernel must be prepared.  Returns
    (grad_in, grad_w)."""
    if not _rows_ok(g) or g.dtype != torch.float32:
        raise ValueError("g must be float32 [nbeam][ndm][nsamp] with 16-byte aligned rows")
    nb, nd, ns = g.shape
    if nd != plan.ndm:
        raise ValueError(f"gradient has {nd} DM rows, plan has {plan.ndm}")
    if x is not None and (not _rows_ok(x) or x.dtype != torch.float32 or tuple(x.shape[:2]) != (nb, plan.nchan)):
        raise ValueError("x must be float32 [nbeam][nchan][>= nin] with 16-byte aligned rows")
    if grad_in is not None and (not _rows_ok(grad_in) or grad_in.dtype != torch.float32
                                or tuple(grad_in.shape) != (nb, plan.nchan, nin)):
        raise ValueError("grad_in must be float32 [nbeam][nchan][nin] with 16-byte aligned rows")
    if grad_w is not None and (grad_w.dtype != torch.float32 or grad_w.numel() != plan.nchan
                               or not grad_w.is_contiguous()):
        raise ValueError("grad_w must be a contiguous float32 tensor of nchan values")
    if w is not None and (w.dtype != torch.float32 or w.numel() != plan.nchan or not w.is_contiguous()):
        raise ValueError("w must be a contiguous float32 tensor of nchan values")
    check(lib().dedisp_adjoint_noalloc(plan.handle, nb, ns, nin, ctypes.c_void_p(g.data_ptr()), g.stride(1),
                                       ctypes.c_void_p(w.data_ptr()) if w is not None else None,
                                       ctypes.c_void_p(x.data_ptr()) if x is not None else None,
                                       x.stride(1) if x is not None else 0,
                                       ctypes.c_void_p(grad_in.data_ptr()) if grad_in is not None else None,
                                       grad_in.stride(1) if grad_in is not None else 0,
                                       ctypes.c_void_p(grad_w.data_ptr()) if grad_w is not None else None,
                                       _stream(g.device)), "adjoint_noalloc")
    return grad_in, grad_w


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _det_outputs(shape, device):
    return {"snr": torch.empty(shape, dtype=torch.float64, device=device),
            "width": torch.empty(shape, dtype=torch.int32, device=device),
            "start": torch.empty(shape, dtype=torch.int32, device=device),
            "mean": torch.empty(shape, dtype=torch.float64, device=device),
            "std": torch.empty(shape, dtype=torch.float64, device=device)}


def detect(x: torch.Tensor, plan: Plan, nsamp: int | None = None, w: torch.Tensor | None = None, nwidth: int = 6,
           workspace: torch.Tensor | None = None) -> dict:
    """Single-pulse search over every dedispersed series without storing the
    series: boxcars of widths 1, 2, ..., 2^(nwidth-1); returns tensors
    [nbeam][ndm] (or [ndm] for 2-D input): snr (f64), width, start (i32),
    mean, std (f64).  See dedisp_detect in include/dedisp.h."""
    squeeze = x.dim() == 2
    xr = _as_rows(x)
    nb, nc, nin = xr.shape
    if nc != plan.nchan:
        raise ValueError(f"input has {nc} channels, plan has {plan.nchan}")
    if nsamp is None:
        nsamp = nin - plan.max_delay
    if nsamp < 1 or nin < nsamp + plan.max_delay:
        raise ValueError(f"need nin >= nsamp + max_delay ({nsamp} + {plan.max_delay}), got {nin}")
    dt = _dt(xr.dtype)
    if w is not None:
        if dt == U8:
            raise ValueError("weights are not supported for uint8 input")
        w = w.detach().to(torch.float32).contiguous()
        if w.numel() != nc or not w.is_cuda:
            raise ValueError("weights must be a float32 GPU tensor of nchan values")
    L = lib()
    nbytes = L.dedisp_detect_workspace_bytes(plan.handle, dt, nb, nsamp)
    if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
        workspace = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=xr.device)
    o = _det_outputs((nb, plan.ndm), xr.device)
    check(L.dedisp_detect(plan.handle, nb, nsamp, _ptr(xr), dt, xr.stride(1), _ptr(w), nwidth, _ptr(o["snr"]),
                          _ptr(o["width"]), _ptr(o["start"]), _ptr(o["mean"]), _ptr(o["std"]), _ptr(workspace),
                          workspace.numel() * workspace.element_size(), _stream(xr.device)), "detect")
    return {k: v[0] for k, v in o.items()} if squeeze else o


def detect_rows(rows: torch.Tensor, nsamp: int | None = None, nwidth: int = 6) -> dict:
    """The same search over stored series rows [..., n] (float32, or int32
    searched in float32); returns tensors of the leading shape."""
    lead = tuple(rows.shape[:-1])
    r = _as_rows(rows.reshape(1, -1, rows.shape[-1]))
    if r.dtype == torch.float32:
        dt = F32
    elif r.dtype == torch.int32:
        dt = I32
    else:
        raise ValueError("rows must be float32 or int32")
    nrows, n = r.shape[1], r.shape[2]
    nsamp = n if nsamp is None else nsamp
    if nsamp < 1 or nsamp > n:
        raise ValueError("need 1 <= nsamp <= row length")
    L = lib()
    nbytes = L.dedisp_detect_rows_workspace_bytes(nrows, nsamp)
    ws = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=r.device)
    o = _det_outputs((nrows,), r.device)
    check(L.dedisp_detect_rows(nrows, nsamp, _ptr(r), dt, r.stride(1), nwidth, _ptr(o["snr"]), _ptr(o["width"]),
                               _ptr(o["start"]), _ptr(o["mean"]), _ptr(o["std"]), _ptr(ws), nbytes,
                               _stream(r.device)), "detect_rows")
    return {k: v.reshape(lead) for k, v in o.items()}


class DedispFunction(torch.autograd.Function):
    """Differentiable dedispersion: forward = dedisperse, backward = adjoint.

    apply(x, w, plan, nsamp) with x [nbeam][nchan][nin] float32 and w [nchan]
    float32 (or None).  Gradients flow to x (gather-form adjoint scaled by w)
    and to w (sum over beams and samples of x times the adjoint)."""

    @staticmethod
    def forward(ctx, x, w, plan, nsamp):
        out = dedisperse(x, plan, w, nsamp)
        ctx.plan = plan
        ctx.nin = x.shape[-1]
        ctx.squeeze = x.dim() == 2
        ctx.save_for_backward(x, w if w is not None else torch.empty(0, device=x.device))
        ctx.has_w = w is not None
        return out

    @staticmethod
    def backward(ctx, g):
        x, w = ctx.saved_tensors
        w = w if ctx.has_w else None
        need_x = ctx.needs_input_grad[0]
        need_w = ctx.has_w and ctx.needs_input_grad[1]
        gi, gw = adjoint(g, ctx.plan, ctx.nin, w, x if need_w else None, want_grad_in=need_x)
        if gi is not None and ctx.squeeze:
            gi = gi[0]
        return gi, gw, None, None


def dedisperse_autograd(x, plan, w=None, nsamp=None):
    if nsamp is None:
        nsamp = x.shape[-1] - plan.max_delay
    return DedispFunction.apply(x, w, plan, nsamp)


def _check_batch_beam(i: int, plan, x, o, nsamp: int, w) -> None:
    """Refuse a batch beam whose buffers do not match its plan.  Runs before
    any library call: the persistent launch sees only pointers, and the
    captured graph keeps them, so nothing may be copied or re-laid out."""
    at = f"beam {i}: "
    if x.dim() != 3 or x.shape[0] != 1 or o.dim() != 3 or o.shape[0] != 1:
        raise ValueError(at + "inputs and outputs are single beams [1][rows][samples]")
    if x.shape[1] != plan.nchan:
        raise ValueError(at + f"input has {x.shape[1]} channels, plan has {plan.nchan}")
    if o.shape[1] != plan.ndm:
        raise ValueError(at + f"output has {o.shape[1]} DM rows, plan has {plan.ndm}")
    if not 1 <= nsamp <= o.shape[2]:
        raise ValueError(at + f"nsamp {nsamp} outside 1..{o.shape[2]} (output row length)")
    if x.shape[2] < nsamp + plan.max_delay:
        raise ValueError(at + f"input rows hold {x.shape[2]} samples, need nsamp + max_delay = "
                         f"{nsamp + plan.max_delay}")
    if x.dtype != torch.float32 or o.dtype != torch.float32:
        raise ValueError(at + "batches take float32 input and output")
    if w is not None and (w.dim() != 1 or w.numel() != plan.nchan or w.dtype != torch.float32
                          or w.stride(0) != 1):
        raise ValueError(at + "weights must be a contiguous float32 tensor of nchan values")
    if not _rows_ok(x) or not _rows_ok(o):
        raise ValueError(at + "rows must start on 16-byte boundaries with 16-byte multiple strides "
                         "(allocate them with empty_rows); batches never copy their buffers")
    if not x.is_cuda or not o.is_cuda or (w is not None and not w.is_cuda):
        raise ValueError(at + "input, output and weights must be on the GPU")


class Batch:
    """Many independent beams (each its own plan, sizes and buffers) run as one
    persistent, graph-captured launch (execute) or as a per-beam launch loop
    (execute_per_beam).  Buffers are used in place: the caller may refill them
    between calls, and they must stay alive while the batch exists.

    tune: time the candidate kernel variants on the batch's own buffers and
    keep the fastest (overwrites the outputs); tune_cache: a JSON file in which
    that choice is looked up first and stored afterwards."""

    def __init__(self, plans, inputs, outputs, nsamps=None, weights=None, tune=False, tune_cache=None):
        L = lib()
        n = len(plans)
        if not (len(inputs) == len(outputs) == n) or n < 1:
            raise ValueError("plans, inputs and outputs must have the same non-zero length")
        if weights is not None and len(weights) != n:
            raise ValueError("weights must have one entry per beam")
        xs = [x.unsqueeze(0) if x.dim() == 2 else x for x in inputs]
        os_ = [o.unsqueeze(0) if o.dim() == 2 else o for o in outputs]
        if nsamps is None:
            nsamps = [o.shape[2] for o in os_]
        for i in range(n):
            _check_batch_beam(i, plans[i], xs[i], os_[i], int(nsamps[i]),
                              None if weights is None else weights[i])
        self._keep = (plans, xs, os_, weights)
        arr = lambda typ, vals: (typ * n)(*vals)  # noqa: E731
        hp = arr(ctypes.c_void_p, [p.handle.value for p in plans])
        ns = arr(ctypes.c_int32, [int(v) for v in nsamps])
        din = arr(ctypes.c_void_p, [x.data_ptr() for x in xs])
        ist = arr(ctypes.c_int64, [x.stride(1) for x in xs])
        dw = arr(ctypes.c_void_p, [w.data_ptr() for w in weights]) if weights is not None else None
        dout = arr(ctypes.c_void_p, [o.data_ptr() for o in os_])
        ost = arr(ctypes.c_int64, [o.stride(1) for o in os_])
        h = ctypes.c_void_p()
        check(L.dedisp_batch_create(ctypes.byref(h), n, hp, ns, din, F32, ist, dw, dout, ost, int(bool(tune)),
                                    tune_cache.encode() if tune_cache else None), "batch_create")
        self._h = h

    @property
    def cache_hit(self) -> bool:
        """True if the variant came from the tune cache (no search ran)."""
        return int(lib().dedisp_batch_cache_hit(self._h)) == 1

    def execute(self):
        check(lib().dedisp_execute_batched(self._h, _stream()), "execute_batched")

    def execute_per_beam(self):
        check(lib().dedisp_execute_per_beam(self._h, _stream()), "execute_per_beam")

    @property
    def variant(self) -> int:
        """Index of the FP32 tiled variant the batch runs."""
        return int(lib().dedisp_batch_variant(self._h))

    @property
    def queues(self) -> int:
        """Work queues of the persistent launch (1, or 8: one per XCD)."""
        return int(lib().dedisp_batch_queues(self._h))

    def set_queues(self, n: int):
        """Rebuild the work table with n (1 or 8) queues, keeping the variant."""
        check(lib().dedisp_batch_set_queues(self._h, int(n)), "batch_set_queues")

    def set_variant(self, i: int):
        """Run the batch with FP32 tiled variant i (rebuilds its work table)."""
        check(lib().dedisp_batch_set_variant(self._h, int(i)), "batch_set_variant")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dedisp_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
