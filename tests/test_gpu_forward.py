"""GPU parity of the forward path against the CPU oracle (Algorithm 1).

FP32: the kernels sum channels in ascending order with one rounding per
term, exactly as the oracle does, so results are expected bit-identical;
the pass gate is |gpu - oracle| <= 1e-5 * sum_c |w_c x_c| per element.
uint8 -> int32: bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _dd():
    import paper_1601_01165_amd as dd

    return dd


def _note(msg):
    print(msg, flush=True)


def _to_gpu(x: np.ndarray, pad_extra: int = 0):
    dd = _dd()
    x3 = x if x.ndim == 3 else x[None]
    dtype = torch.uint8 if x3.dtype == np.uint8 else torch.float32
    t = dd.empty_rows(x3.shape[0], x3.shape[1], x3.shape[2] + pad_extra, dtype, "cuda", zero=True)
    t = t[:, :, : x3.shape[2]]
    t.copy_(torch.from_numpy(np.ascontiguousarray(x3)))
    return t


def _check_f32(got: np.ndarray, x: np.ndarray, delta: np.ndarray, nsamp: int, w=None, where=""):
    ref = oracle.forward_f32(x, delta, nsamp, w)
    _, scale = oracle.forward_f64(x.astype(np.float64), delta, nsamp,
                                  None if w is None else w.astype(np.float64), with_scale=True)
    err = np.abs(got.astype(np.float64) - ref.astype(np.float64))
    bad = err > TOL * scale + 1e-30
    assert not bad.any(), f"{where}: {int(bad.sum())} elements over tolerance, max err {err.max()}"
    same = float(np.mean(got == ref))
    _note(f"{where}: bit-identical fraction {same:.6f}")
    assert same == 1.0, f"{where}: expected bit-identical FP32 (ascending channels, one rounding per term)"


def _variants(plan, dtype):
    dd = _dd()
    out = [-1]
    for i in range(len(dd.variant_names(dtype))):
        try:
            plan.set_variant(i, dtype)
            out.append(i)
        except dd.DedispError:
            pass
    return out


def test_plan_delays_match_oracle():
    dd = _dd()
    for k in (0, 1, 2):
        b = synth.config(k)[0]
        _note(f"plan delays config {k}")
        p = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
        ref = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
        assert np.array_equal(p.delays(), ref)
        assert p.max_delay == int(ref.max())


def test_config0_all_variants():
    dd = _dd()
    b = synth.config(0)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    x = synth.noise(b, nin)
    for j, t0 in synth.pulses(b, int(delta.max())):
        synth.inject(x, delta, j, t0, b.pulse_width, b.pulse_amp)
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    xg = _to_gpu(x)
    vs = _variants(plan, "f32")
    assert len(vs) >= 3
    for v in vs:
        _note(f"config0 variant {v}")
        plan.set_variant(v)
        out = dd.dedisperse(xg, plan, nsamp=b.nsamp)
        torch.cuda.synchronize()
        _check_f32(out.cpu().numpy(), x, delta, b.nsamp, where=f"config0 v{v}")
    # the injected pulse is recovered at its DM
    out = out.cpu().numpy()[0]
    snr = [oracle.snr(out[j]) for j in range(b.ndm)]
    assert int(np.argmax(snr)) == 17


def test_config0_weighted():
    dd = _dd()
    b = synth.config(0)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, b.nchan, nin)).astype(np.float32)
    w = rng.uniform(0.25, 2.0, b.nchan).astype(np.float32)
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    xg = _to_gpu(x)
    wg = torch.from_numpy(w).cuda()
    for v in _variants(plan, "f32"):
        _note(f"config0 weighted variant {v}")
        plan.set_variant(v)
        out = dd.dedisperse(xg, plan, wg, nsamp=b.nsamp)
        torch.cuda.synchronize()
        _check_f32(out.cpu().numpy(), x, delta, b.nsamp, w, where=f"weighted v{v}")


CASES = [
    # nchan, ndm, nsamp, nbeam, band (lo, hi), tsamp, dm step, order
    (1, 1, 1, 1, (1400, 1500), 5e-5, 1.0, "asc"),
    (1, 7, 300, 2, (1400, 1500), 5e-5, 1.0, "asc"),
    (3, 1, 1025, 1, (1400, 1500), 5e-5, 2.0, "asc"),
    (17, 33, 513, 1, (1270, 1570), 5e-5, 0.25, "desc"),
    (64, 70, 1500, 3, (1270, 1570), 5e-5, 0.25, "asc"),
    (130, 45, 2049, 1, (1270, 1570), 5e-5, 0.25, "shuffled"),
    (200, 97, 3000, 1, (300, 400), 1e-4, 0.1, "dup"),
]


@pytest.mark.parametrize("case", CASES, ids=[f"c{c[0]}_d{c[1]}_s{c[2]}_b{c[3]}_{c[7]}" for c in CASES])
def test_ragged_shapes(case):
    dd = _dd()
    nc, nd, ns, nb, (lo, hi), ts, step, order = case
    rng = np.random.default_rng(nc * 1000 + nd)
    f = lo + (np.arange(nc) + 0.5) * (hi - lo) / nc
    dms = np.arange(nd) * step
    if order == "desc":
        f = f[::-1].copy()
    elif order == "shuffled":
        dms = rng.permutation(dms)
    elif order == "dup":
        dms[5:9] = dms[5]
        dms = rng.permutation(dms)
    delta = oracle.delay_table(f, ts, dms)
    nin = ns + int(delta.max()) + 3
    x = rng.standard_normal((nb, nc, nin)).astype(np.float32)
    plan = dd.Plan(f, ts, dms)
    xg = _to_gpu(x, pad_extra=5)
    for v in _variants(plan, "f32"):
        _note(f"ragged {case} variant {v}")
        plan.set_variant(v)
        out = dd.dedisperse(xg, plan, nsamp=ns)
        torch.cuda.synchronize()
        _check_f32(out.cpu().numpy(), x, delta, ns, where=f"{case} v{v}")


def test_u8_small_all_variants():
    dd = _dd()
    b = synth.config(2)[0]
    dms = b.dms()[:300]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, dms)
    ns = 5000
    nin = ns + int(delta.max())
    rng = np.random.default_rng(7)
    x = rng.integers(0, 256, size=(2, b.nchan, nin)).astype(np.uint8)
    ref = oracle.forward_u8(x, delta, ns)
    plan = dd.Plan(b.freqs(), b.tsamp_s, dms)
    xg = _to_gpu(x)
    vs = _variants(plan, "u8")
    assert len(vs) >= 2
    for v in vs:
        _note(f"u8 variant {v}")
        plan.set_variant(v, "u8")
        out = dd.dedisperse(xg, plan, nsamp=ns)
        torch.cuda.synchronize()
        assert out.dtype == torch.int32
        assert np.array_equal(out.cpu().numpy(), ref), f"u8 variant {v} differs"


def test_u8_ragged():
    dd = _dd()
    rng = np.random.default_rng(9)
    for nc, nd, ns in [(1, 1, 1), (5, 3, 17), (32, 41, 1031), (40, 9, 4097)]:
        f = 134.875 + (np.arange(nc) + 0.5) * 6.25 / nc
        dms = rng.permutation(np.arange(nd) * 0.01)
        delta = oracle.delay_table(f, 5e-6, dms)
        nin = ns + int(delta.max())
        x = rng.integers(0, 256, size=(1, nc, nin)).astype(np.uint8)
        ref = oracle.forward_u8(x, delta, ns)
        plan = dd.Plan(f, 5e-6, dms)
        xg = _to_gpu(x, pad_extra=16)
        for v in _variants(plan, "u8"):
            _note(f"u8 ragged {(nc, nd, ns)} variant {v}")
            plan.set_variant(v, "u8")
            out = dd.dedisperse(xg, plan, nsamp=ns)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref), (nc, nd, ns, v)


@pytest.mark.parametrize("nc", [256, 257, 600])
def test_u8_many_rows_packed_sums(nc):
    """Sums past 16 bits: 256 rows of 255 are the most the packed sums of the
    byte-shifted variants hold (the shifted-dword sum stays below 2^32); 257
    and 600 rows need the int32 flush of the wide variants (the narrow ones
    must refuse such plans)."""
    dd = _dd()
    rng = np.random.default_rng(nc)
    f = 1270.0 + (np.arange(nc) + 0.5) * 300.0 / nc
    dms = np.arange(24) * 0.25
    delta = oracle.delay_table(f, 50e-6, dms)
    ns = 1500
    nin = ns + int(delta.max())
    x = np.full((1, nc, nin), 255, np.uint8)
    x[:, ::3] = rng.integers(200, 256, size=x[:, ::3].shape).astype(np.uint8)
    ref = oracle.forward_u8(x, delta, ns)
    plan = dd.Plan(f, 50e-6, dms)
    names = dd.variant_names("u8")
    vs = _variants(plan, "u8")
    narrow = [i for i, n in enumerate(names) if n.startswith("u8s_") and not n.endswith("_wide")]
    wide = [i for i, n in enumerate(names) if n.endswith("_wide")]
    assert wide and all(v in vs for v in wide)
    if nc > 256:
        assert not any(v in vs for v in narrow)
    else:
        assert all(v in vs for v in narrow)
    xg = _to_gpu(x, pad_extra=16)
    for v in vs:
        _note(f"u8 {nc} rows variant {v}")
        plan.set_variant(v, "u8")
        out = dd.dedisperse(xg, plan, nsamp=ns)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), (nc, v)


def _sample_points(rng, nb, nd, ns, n):
    pb = rng.integers(0, nb, n)
    pd = rng.integers(0, nd, n)
    ps = rng.integers(0, ns, n)
    # always include the edges
    pb = np.concatenate([pb, [0, nb - 1, nb - 1]])
    pd = np.concatenate([pd, [0, nd - 1, nd - 1]])
    ps = np.concatenate([ps, [0, ns - 1, 0]])
    return pb, pd, ps


def test_config1_full_size_sampled():
    """Apertif-like beam at full size with the default (benchmarked) kernel."""
    dd = _dd()
    b = synth.config(1)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    _note("config1: generating input")
    x = synth.noise(b, nin, synth.padded_len(nin, 4))
    for j, t0 in synth.pulses(b, int(delta.max())):
        synth.inject(x, delta, j, t0, b.pulse_width, b.pulse_amp)
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    _note(f"config1 default variant {plan.variant()}")
    # untuned, the plan takes the measured-fastest shape that fits this geometry
    assert dd.variant_names("f32")[plan.variant()] == "win_tp20_dpw4_nw16_win40_cc10_buf2_jmp"
    xg = torch.from_numpy(x).cuda()[None][:, :, :nin]
    out = dd.dedisperse(xg, plan, nsamp=b.nsamp)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    rng = np.random.default_rng(11)
    pb, pd, ps = _sample_points(rng, 1, b.ndm, b.nsamp, 20000)
    ref, scale = oracle.forward_points(np.ascontiguousarray(x[None, :, :nin]), delta, pb, pd, ps)
    got = o[pb, pd, ps]
    assert (np.abs(got.astype(np.float64) - ref) <= TOL * scale).all()
    assert np.array_equal(got, ref)
    # whole rows at the pulse DMs and the last DM
    rows = sorted({j for j, _ in synth.pulses(b, int(delta.max()))} | {b.ndm - 1})
    full = oracle.forward_f32(np.ascontiguousarray(x[None, :, :nin]), delta[rows], b.nsamp)
    assert np.array_equal(o[0, rows], full[0])


def test_config2_full_size_sampled():
    """LOFAR-like uint8 beam at full size (bit-exact)."""
    dd = _dd()
    b = synth.config(2)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    _note("config2: generating input")
    x = synth.noise(b, nin, synth.padded_len(nin, 1))
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    _note(f"config2 default u8 variant {plan.variant('u8')}")
    assert dd.variant_names("u8")[plan.variant("u8")] == "u8s_q4_dpw4_nw16_cc4_o8"
    xg = torch.from_numpy(x).cuda()[None][:, :, :nin]
    out = dd.dedisperse(xg, plan, nsamp=b.nsamp)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    rng = np.random.default_rng(12)
    pb, pd, ps = _sample_points(rng, 1, b.ndm, b.nsamp, 50000)
    ref, _ = oracle.forward_points(np.ascontiguousarray(x[None, :, :nin]), delta, pb, pd, ps)
    assert np.array_equal(o[pb, pd, ps], ref)
    rows = [0, 1, 1000, b.ndm - 1]
    full = oracle.forward_u8(np.ascontiguousarray(x[None, :, :nin]), delta[rows], b.nsamp)
    assert np.array_equal(o[0, rows], full[0])


def test_errors_on_gpu():
    dd = _dd()
    from paper_1601_01165_amd import _clib

    b = synth.config(0)[0]
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    x = dd.empty_rows(1, b.nchan, b.nsamp + plan.max_delay, torch.float32, "cuda", zero=True)
    out = dd.empty_rows(1, b.ndm, b.nsamp, torch.float32, "cuda")
    L = dd.lib()
    s = None
    # stride too small
    st = L.dedisp_execute(plan.handle, 1, b.nsamp, x.data_ptr(), _clib.F32, b.nsamp, None, out.data_ptr(), _clib.F32,
                          out.stride(1), s)
    assert st == _clib.E_SHAPE
    # misaligned row
    st = L.dedisp_execute(plan.handle, 1, b.nsamp, x.data_ptr(), _clib.F32, x.stride(1) - 1, None, out.data_ptr(),
                          _clib.F32, out.stride(1), s)
    assert st in (_clib.E_ALIGN, _clib.E_SHAPE)
    st = L.dedisp_execute(plan.handle, 1, b.nsamp, x.data_ptr() + 4, _clib.F32, x.stride(1), None, out.data_ptr(),
                          _clib.F32, out.stride(1), s)
    assert st == _clib.E_ALIGN
    # dtype pair
    st = L.dedisp_execute(plan.handle, 1, b.nsamp, x.data_ptr(), _clib.U8, x.stride(1) * 4, None, out.data_ptr(),
                          _clib.F32, out.stride(1), s)
    assert st == _clib.E_DTYPE
    # weights with uint8
    st = L.dedisp_execute(plan.handle, 1, b.nsamp, x.data_ptr(), _clib.U8, x.stride(1) * 4, x.data_ptr(),
                          out.data_ptr(), _clib.I32, out.stride(1), s)
    assert st == _clib.E_DTYPE
    assert L.dedisp_plan_set_variant(plan.handle, _clib.F32, 999) == _clib.E_INVALID
    # empty and oversized calls are refused before any launch
    args = (x.data_ptr(), _clib.F32, x.stride(1), None, out.data_ptr(), _clib.F32, out.stride(1), s)
    assert L.dedisp_execute(plan.handle, 1, 0, *args) == _clib.E_INVALID
    assert L.dedisp_execute(plan.handle, 0, b.nsamp, *args) == _clib.E_INVALID
    assert L.dedisp_execute(plan.handle, 65536, b.nsamp, *args) == _clib.E_SHAPE
    assert L.dedisp_execute(plan.handle, 1, b.nsamp, None, *args[1:]) == _clib.E_INVALID
    assert L.dedisp_execute(plan.handle, 1, b.nsamp, x.data_ptr(), _clib.F32, (1 << 29) + 4, None, out.data_ptr(),
                            _clib.F32, out.stride(1), s) == _clib.E_SHAPE
    g = dd.empty_rows(1, b.ndm, b.nsamp, torch.float32, "cuda", zero=True)
    nin = b.nsamp + plan.max_delay
    gi = dd.empty_rows(1, b.nchan, nin, torch.float32, "cuda")
    assert L.dedisp_adjoint(plan.handle, 65536, b.nsamp, nin, g.data_ptr(), g.stride(1), None, None, 0,
                            gi.data_ptr(), gi.stride(1), None, None, 0, s) == _clib.E_SHAPE
    torch.cuda.synchronize()


def _seq_channel_sum(x2, ns, w=None):
    """Sequential FP32 sum over channels (ascending, one rounding per term),
    written independently of the oracle: the value every DM-0 output takes."""
    acc = np.zeros(ns, np.float32)
    for c in range(x2.shape[0]):
        term = x2[c, :ns] if w is None else (w[c] * x2[c, :ns]).astype(np.float32)
        acc = (acc + term).astype(np.float32)
    return acc


@pytest.mark.parametrize("weighted", [False, True])
def test_perfect_reuse_all_zero_dms_f32(weighted):
    """The perfect-reuse set-up of Section 4.3: every DM trial is 0, so every
    delay span is 0 and every trial reads the same samples.  Every FP32
    variant and the direct kernel, against the oracle bit for bit, and every
    row equal to the sequential channel sum.  Weights are powers of two so
    that w * x is exact and the weighted sum is still a sequential FP32 sum."""
    dd = _dd()
    b = synth.config(1)[0]
    f = b.freqs()[::4]  # 256 channels of the Apertif-like band
    ns, nd = 2049, 97
    dms = np.zeros(nd)
    delta = oracle.delay_table(f, b.tsamp_s, dms)
    assert (delta == 0).all()
    rng = np.random.default_rng(81)
    x = rng.standard_normal((2, f.size, ns + 3)).astype(np.float32)
    w = (2.0 ** rng.integers(-2, 3, f.size)).astype(np.float32) if weighted else None
    plan = dd.Plan(f, b.tsamp_s, dms)
    assert plan.max_delay == 0
    xg = _to_gpu(x)
    wg = torch.from_numpy(w).cuda() if weighted else None
    rows = [_seq_channel_sum(x[k], ns, w) for k in range(2)]
    vs = _variants(plan, "f32")
    assert len(vs) == len(dd.variant_names("f32")) + 1  # zero spans fit every variant
    for v in vs:
        _note(f"perfect reuse f32 variant {v} weighted={weighted}")
        plan.set_variant(v)
        out = dd.dedisperse(xg, plan, wg, nsamp=ns)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        _check_f32(got, x, delta, ns, w, where=f"perfect reuse v{v}")
        for k in range(2):
            assert (got[k] == rows[k][None, :]).all(), (v, k)


def test_perfect_reuse_and_dm_runs_u8():
    """uint8: all-zero DM trials (every row the integer channel sum) and a DM
    list made of long runs of equal values (equal trials give equal rows),
    every uint8 variant and the direct kernel, bit-exact against the oracle."""
    dd = _dd()
    b = synth.config(2)[0]
    ns = 3001
    rng = np.random.default_rng(83)
    runs = np.concatenate([np.zeros(40), np.full(25, 0.5), np.full(31, 0.51), np.full(9, 3.0),
                           np.arange(12) * 0.01 + 1.0, np.full(20, 1.11)])
    for name, dms in (("zero", np.zeros(64)), ("runs", runs)):
        delta = oracle.delay_table(b.freqs(), b.tsamp_s, dms)
        nin = ns + int(delta.max())
        x = rng.integers(0, 256, size=(1, b.nchan, nin)).astype(np.uint8)
        ref = oracle.forward_u8(x, delta, ns)
        plan = dd.Plan(b.freqs(), b.tsamp_s, dms)
        xg = _to_gpu(x, pad_extra=16)
        chan_sum = x[0, :, :ns].astype(np.int64).sum(axis=0)
        for v in _variants(plan, "u8"):
            _note(f"u8 {name} variant {v}")
            plan.set_variant(v, "u8")
            out = dd.dedisperse(xg, plan, nsamp=ns)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            assert np.array_equal(got, ref), (name, v)
            if name == "zero":
                assert (got[0] == chan_sum[None, :]).all(), v
            for j in range(1, dms.size):
                if dms[j] == dms[j - 1]:
                    assert np.array_equal(got[0, j], got[0, j - 1]), (name, v, j)


def test_dm_runs_f32():
    """FP32 with a DM list of long runs of equal trials (and a few isolated
    ones): every variant bit for bit against the oracle, equal trials equal."""
    dd = _dd()
    b = synth.config(1)[0]
    f = b.freqs()[::8]
    runs = np.concatenate([np.zeros(33), np.full(40, 12.25), np.array([12.5, 13.0]), np.full(27, 100.0),
                           np.full(5, 100.25), np.full(21, 300.0)])
    delta = oracle.delay_table(f, b.tsamp_s, runs)
    ns = 1800
    rng = np.random.default_rng(85)
    x = rng.standard_normal((1, f.size, ns + int(delta.max()))).astype(np.float32)
    plan = dd.Plan(f, b.tsamp_s, runs)
    xg = _to_gpu(x)
    for v in _variants(plan, "f32"):
        _note(f"dm runs f32 variant {v}")
        plan.set_variant(v)
        out = dd.dedisperse(xg, plan, nsamp=ns)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        _check_f32(got, x, delta, ns, where=f"dm runs v{v}")
        for j in range(1, runs.size):
            if runs[j] == runs[j - 1]:
                assert np.array_equal(got[0, j], got[0, j - 1]), (v, j)
