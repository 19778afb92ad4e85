"""CPU checks of the C-ABI library: it loads, exports every declared entry
point, and its host-side delay table equals the oracle's (two independent
implementations of Section 2, Equation 1).  No GPU work is done here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(dedisp_[a-z_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def clib():
    from paper_1601_01165_amd import _clib

    return _clib.load()


def test_every_declared_symbol_is_exported(clib):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(clib, n), n
    from paper_1601_01165_amd import _clib

    assert set(names) == set(_clib.SIGNATURES), "binding and header disagree"


def test_status_strings(clib):
    for s in range(9):
        assert clib.dedisp_status_string(s)
    assert clib.dedisp_status_string(99) == b"unknown status"


def test_variant_names(clib):
    import paper_1601_01165_amd as dd

    f = dd.variant_names("f32")
    u = dd.variant_names("u8")
    assert len(f) >= 4 and len(u) >= 3
    assert len(set(f)) == len(f) and len(set(u)) == len(u)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_host_delays_equal_oracle(k):
    import paper_1601_01165_amd as dd

    beams = synth.config(k)
    seen = set()
    for b in beams[:12]:
        key = (b.nchan, b.ndm)
        if key in seen:
            continue
        seen.add(key)
        got = dd.compute_delays(b.freqs(), b.tsamp_s, b.dms())
        ref = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
        assert np.array_equal(got, ref)


def test_host_delays_any_order_and_duplicates():
    import paper_1601_01165_amd as dd

    rng = np.random.default_rng(3)
    f = rng.uniform(300, 400, 37)
    dms = np.concatenate([rng.uniform(0, 100, 20), [5.0, 5.0, 0.0]])
    assert np.array_equal(dd.compute_delays(f, 1e-4, dms), oracle.delay_table(f, 1e-4, dms))


def test_host_delays_errors(clib):
    import paper_1601_01165_amd as dd
    from paper_1601_01165_amd import _clib

    cases = [
        (([1400.0], 0.0, [1.0]), _clib.E_INVALID),
        (([1400.0, -1.0], 1e-3, [1.0]), _clib.E_INVALID),
        (([1400.0], 1e-3, [-1.0]), _clib.E_INVALID),
        (([1400.0, float("nan")], 1e-3, [1.0]), _clib.E_INVALID),
        (([1400.0], 1e-3, [float("inf")]), _clib.E_INVALID),
        (([1.0, 1e9], 1e-9, [1e6]), _clib.E_SHAPE),
    ]
    for args, code in cases:
        with pytest.raises(dd.DedispError) as ei:
            dd.compute_delays(*args)
        assert ei.value.status == code, args
    out = np.empty(4, np.int32)
    f = np.array([1.0, 2.0])
    assert clib.dedisp_compute_delays(0, f.ctypes.data, 1.0, 1, f.ctypes.data, out.ctypes.data, None) == _clib.E_INVALID
    assert clib.dedisp_compute_delays(2, None, 1.0, 1, f.ctypes.data, out.ctypes.data, None) == _clib.E_INVALID


def test_null_handles_are_rejected(clib):
    from paper_1601_01165_amd import _clib

    assert clib.dedisp_plan_destroy(None) == _clib.OK
    assert clib.dedisp_batch_destroy(None) == _clib.OK
    assert clib.dedisp_plan_info(None, None, None, None) == _clib.E_INVALID
    assert clib.dedisp_execute(None, 1, 1, None, 0, 1, None, None, 0, 1, None) == _clib.E_INVALID
    assert clib.dedisp_adjoint(None, 1, 1, 1, None, 1, None, None, 0, None, 0, None, None, 0, None) == _clib.E_INVALID
    assert clib.dedisp_execute_batched(None, None) == _clib.E_INVALID
    assert clib.dedisp_plan_create(None, 1, None, 1.0, 1, None) == _clib.E_INVALID
    h = ctypes.c_void_p()
    f = np.array([1400.0])
    assert clib.dedisp_plan_create(ctypes.byref(h), 0, f.ctypes.data, 1.0, 1, f.ctypes.data) == _clib.E_INVALID
    assert not h.value


def test_detect_argument_checks(clib):
    # every check below fails before any device work
    from paper_1601_01165_amd import _clib

    E = _clib
    assert clib.dedisp_detect(None, 1, 1, None, 0, 1, None, 6, None, None, None, None, None, None, 0, None) == E.E_INVALID
    assert clib.dedisp_detect_workspace_bytes(None, 0, 1, 1) == 0
    assert clib.dedisp_detect_variant(None, 0) == -1
    assert clib.dedisp_detect_rows_workspace_bytes(0, 10) == 0
    # 3 rows of 2000 samples: two 992-start tiles and a partial one, 64-byte records
    assert clib.dedisp_detect_rows_workspace_bytes(3, 2000) == 3 * 3 * 64
    p = ctypes.c_void_p(4096)  # never dereferenced: the checks fail first
    def rows(n, ns, dt, stride, nw, snr=p, ws=p, wsb=1 << 20, rowp=p):
        return clib.dedisp_detect_rows(n, ns, rowp, dt, stride, nw, snr, p, p, None, None, ws, wsb, None)
    assert rows(0, 10, E.F32, 12, 6) == E.E_INVALID
    assert rows(2, 0, E.F32, 12, 6) == E.E_INVALID
    assert rows(2, 10, E.F32, 12, 6, rowp=None) == E.E_INVALID
    assert rows(2, 10, E.F32, 12, 0) == E.E_INVALID
    assert rows(2, 10, E.F32, 12, 7) == E.E_INVALID
    assert rows(2, 10, E.F32, 12, 6, snr=None) == E.E_INVALID
    assert rows(2, 10, E.U8, 16, 6) == E.E_DTYPE
    assert rows(2, 10, E.F32, 8, 6) == E.E_SHAPE
    assert rows(2, 10, E.F32, 10, 6) == E.E_ALIGN
    assert rows(2, 10, E.F32, 12, 6, rowp=ctypes.c_void_p(4100)) == E.E_ALIGN
    assert rows(2, 10, E.F32, 12, 6, ws=None) == E.E_WORKSPACE
    assert rows(2, 10, E.F32, 12, 6, ws=ctypes.c_void_p(4104)) == E.E_ALIGN
    assert rows(2, 10, E.F32, 12, 6, wsb=64) == E.E_WORKSPACE


class _FakePlan:
    """Stand-in for a Plan (the batch checks read only its sizes)."""

    nchan, ndm, max_delay = 8, 5, 30


def _aligned(shape, dtype="float32"):
    import torch

    dt = getattr(torch, dtype)
    es = torch.empty((), dtype=dt).element_size()
    q = 16 // es
    n = (shape[2] + q - 1) // q * q
    return torch.zeros((shape[0], shape[1], n), dtype=dt)[:, :, : shape[2]]


def test_batch_beam_checks_refuse_before_any_launch():
    """Every mismatch between a batch beam's buffers and its plan is refused
    on the host, before the library sees the pointers."""
    import torch

    import paper_1601_01165_amd as dd

    p = _FakePlan()
    x = _aligned((1, 8, 130))
    o = _aligned((1, 5, 100))
    chk = dd._check_batch_beam
    cases = [
        ((_aligned((1, 7, 130)), o, 100, None), "channels"),
        ((x, _aligned((1, 6, 100)), 100, None), "DM rows"),
        ((x, o, 101, None), "nsamp"),
        ((x, o, 0, None), "nsamp"),
        ((_aligned((1, 8, 129)), o, 100, None), "max_delay"),
        ((_aligned((1, 8, 130), "uint8"), o, 100, None), "float32"),
        ((x, _aligned((1, 5, 100), "int32"), 100, None), "float32"),
        ((x, o, 100, torch.ones(7)), "weights"),
        ((x, o, 100, torch.ones(8, dtype=torch.float64)), "weights"),
        ((torch.zeros((1, 8, 131))[:, :, :130], o, 100, None), "16-byte"),   # row stride 131 floats
        ((x, torch.zeros((1, 5, 101))[:, :, :100], 100, None), "16-byte"),
        ((torch.zeros((1, 8, 133))[:, :, 1:131], o, 100, None), "16-byte"),  # base off by 4 bytes
        ((x, o, 100, None), "GPU"),                                          # right shapes, host memory
        ((x, o, 100, torch.ones(8)), "GPU"),
    ]
    for args, what in cases:
        with pytest.raises(ValueError, match=what):
            chk(0, p, *args)
