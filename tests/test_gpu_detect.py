"""GPU parity of the single-pulse search (boxcar S/N over every dedispersed
series) against the oracle's FP64 search of the oracle's dedispersed rows.

uint8 input: the series and boxcar sums are exact integers on both sides, so
widths and starts must match exactly; S/N, mean and std agree to FP64
rounding (relative 1e-10; the moments are one-pass on the GPU, two-pass in
the oracle).  The width decision compares S/N values in FP64 on both sides;
where two widths score within 1e-10 of each other either choice is valid.

float32 input: the GPU series equal the oracle's bit for bit (the forward
parity tests check that); the GPU boxcar sums are FP32 pairwise doublings
(at most log2(w) <= 5 roundings of partial sums), so each sum is within
5 * 2^-24 * sum|y| of the exact one.  The S/N gate per series is
5 * 2^-24 * 32 * max|y| / std + 1e-9 * (1 + |S/N|); the chosen (width, start)
must reach the oracle's best S/N within twice that, and at least 98% of the
series must pick exactly the oracle's window.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _dd():
    import paper_1601_01165_amd as dd

    return dd


def _note(msg):
    print(msg, flush=True)


def _to_gpu(x: np.ndarray):
    dd = _dd()
    x3 = x if x.ndim == 3 else x[None]
    dtype = torch.uint8 if x3.dtype == np.uint8 else torch.float32
    t = dd.empty_rows(x3.shape[0], x3.shape[1], x3.shape[2], dtype, "cuda", zero=True)
    t.copy_(torch.from_numpy(np.ascontiguousarray(x3)))
    return t


def _cpu(res):
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in res.items()}


def _snr_at(y, w, t):
    y = np.asarray(y, np.float64)
    m, s = y.mean(), y.std()
    if s == 0:
        return 0.0
    return (y[t:t + w].sum() - w * m) / (s * np.sqrt(w))


def _check_exact(got, rows, nwidth, where):
    """uint8 path: rows [..., nsamp] int32 from the oracle."""
    ref = oracle.detect(rows, nwidth)
    flat = rows.reshape(-1, rows.shape[-1])
    g = {k: v.reshape(-1) for k, v in got.items()}
    r = {k: v.reshape(-1) for k, v in ref.items()}
    assert np.allclose(g["mean"], r["mean"], rtol=1e-12, atol=0), where
    assert np.allclose(g["std"], r["std"], rtol=1e-10, atol=1e-12), where
    assert np.allclose(g["snr"], r["snr"], rtol=1e-10, atol=1e-12), where
    diff = (g["width"] != r["width"]) | (g["start"] != r["start"])
    for i in np.nonzero(diff)[0]:
        # only a tie between widths may differ; the start must then be that width's first maximum
        w, t = int(g["width"][i]), int(g["start"][i])
        assert abs(_snr_at(flat[i], w, t) - r["snr"][i]) <= 1e-10 * (1 + abs(r["snr"][i])), (where, i)
        b = oracle.boxcar_sums(flat[i], w)
        assert t == int(np.argmax(b)), (where, i)
    _note(f"{where}: {flat.shape[0]} series, {int(diff.sum())} width ties")


def _check_f32(got, rows, nwidth, where, min_exact=0.98):
    ref = oracle.detect(rows, nwidth)
    flat = rows.reshape(-1, rows.shape[-1]).astype(np.float64)
    g = {k: v.reshape(-1) for k, v in got.items()}
    r = {k: v.reshape(-1) for k, v in ref.items()}
    sd = np.maximum(r["std"], 1e-300)
    tol = 5 * U * 32 * np.abs(flat).max(axis=1) / sd + 1e-9 * (1 + np.abs(r["snr"]))
    assert np.allclose(g["mean"], r["mean"], rtol=1e-9, atol=1e-9 * sd.max()), where
    assert np.allclose(g["std"], r["std"], rtol=1e-9, atol=1e-12), where
    err = np.abs(g["snr"] - r["snr"])
    assert (err <= tol).all(), f"{where}: S/N error {err.max()} over gate {tol[np.argmax(err - tol)]}"
    for i in range(flat.shape[0]):
        w, t = int(g["width"][i]), int(g["start"][i])
        assert w >= 1 and 0 <= t <= flat.shape[1] - w, (where, i, w, t)
        assert _snr_at(flat[i], w, t) >= r["snr"][i] - 2 * tol[i], (where, i)
    same = float(np.mean((g["width"] == r["width"]) & (g["start"] == r["start"])))
    _note(f"{where}: {flat.shape[0]} series, exact window fraction {same:.4f}, max S/N error {err.max():.3e}")
    assert same >= min_exact, where


def test_u8_exact_small():
    dd = _dd()
    b = synth.config(2)[0]
    # config-2 channels and DMs, fewer samples: several tiles and a ragged tail
    for ns, nd in ((3001, 64), (993, 40), (5000, 17)):
        dms = b.dms()[:nd]
        delta = oracle.delay_table(b.freqs(), b.tsamp_s, dms)
        nin = ns + int(delta.max())
        rng = np.random.default_rng(ns)
        x = np.clip(np.rint(128 + 16 * rng.standard_normal((2, b.nchan, nin))), 0, 255).astype(np.uint8)
        # a wide pulse on beam 1 at DM 5
        for c in range(b.nchan):
            s = 700 + int(delta[5, c])
            x[1, c, s:s + 8] = np.minimum(255, x[1, c, s:s + 8].astype(int) + 60).astype(np.uint8)
        plan = dd.Plan(b.freqs(), b.tsamp_s, dms)
        xg = _to_gpu(x)
        rows = oracle.forward_u8(x, delta, ns)
        for nw in (1, 3, 6):
            _note(f"u8 nsamp {ns} ndm {nd} nwidth {nw} variant {plan.detect_variant('u8')}")
            got = _cpu(dd.detect(xg, plan, nsamp=ns, nwidth=nw))
            _check_exact(got, rows, nw, f"u8 ns{ns} nd{nd} nw{nw}")
        assert int(np.argmax(got["snr"][1])) == 5 and got["width"][1, 5] == 8 and got["start"][1, 5] == 700


def test_u8_every_fused_variant():
    dd = _dd()
    b = synth.config(2)[0]
    ns, nd = 2500, 96
    dms = b.dms()[:nd]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, dms)
    nin = ns + int(delta.max())
    x = synth.noise(b, nin)[None]
    rows = oracle.forward_u8(x, delta, ns)
    plan = dd.Plan(b.freqs(), b.tsamp_s, dms)
    xg = _to_gpu(x)
    names = dd.variant_names("u8")
    seen = set()
    for i, name in enumerate(names):
        try:
            plan.set_detect_variant(i, "u8")  # refused: no search epilogue, or it does not fit
        except dd.DedispError:
            continue
        assert plan.detect_variant("u8") == i
        seen.add(name)
        _note(f"u8 fused variant {name}")
        _check_exact(_cpu(dd.detect(xg, plan, nsamp=ns)), rows, 6, f"u8 {name}")
    assert len(seen) >= 8, seen


def test_f32_config0_every_fused_variant_and_weights():
    dd = _dd()
    b = synth.config(0)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    x = synth.noise(b, nin)
    for j, t0 in synth.pulses(b, int(delta.max())):
        synth.inject(x, delta, j, t0, b.pulse_width, b.pulse_amp)
    w = np.random.default_rng(9).uniform(0.25, 2.0, b.nchan).astype(np.float32)
    rows = oracle.forward_f32(x[None], delta, b.nsamp)
    rows_w = oracle.forward_f32(x[None], delta, b.nsamp, w)
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    xg = _to_gpu(x)
    wg = torch.from_numpy(w).cuda()
    seen = 0
    for i, name in enumerate(dd.variant_names("f32")):
        try:
            plan.set_detect_variant(i, "f32")  # refused: no search epilogue, or it does not fit
        except dd.DedispError:
            continue
        assert plan.detect_variant("f32") == i
        seen += 1
        _note(f"f32 fused variant {name}")
        got = _cpu(dd.detect(xg, plan, nsamp=b.nsamp))
        _check_f32(got, rows, 6, f"f32 {name}")
        assert int(np.argmax(got["snr"][0])) == 17 and got["width"][0, 17] == 4 and got["start"][0, 17] == 2048
        _check_f32(_cpu(dd.detect(xg, plan, nsamp=b.nsamp, w=wg)), rows_w, 6, f"f32 weighted {name}")
    # config 0's delay steps (5.5 samples per DM at the lowest channel) fit
    # only the 4-DM-per-wave variants; the Apertif-like geometry fits all
    assert seen >= 2
    nc, nd, ns = 256, 96, 3000
    f = 1270.0 + (np.arange(nc) + 0.5) * 300.0 / nc
    dms = np.arange(nd) * 0.25
    delta = oracle.delay_table(f, 5e-5, dms)
    x = np.random.default_rng(4).standard_normal((1, nc, ns + int(delta.max()))).astype(np.float32)
    rows = oracle.forward_f32(x, delta, ns)
    plan = dd.Plan(f, 5e-5, dms)
    xg = _to_gpu(x)
    seen = 0
    for i, name in enumerate(dd.variant_names("f32")):
        try:
            plan.set_detect_variant(i, "f32")  # refused: no search epilogue, or it does not fit
        except dd.DedispError:
            continue
        assert plan.detect_variant("f32") == i
        seen += 1
        _note(f"f32 fused variant {name}, Apertif-like geometry")
        _check_f32(_cpu(dd.detect(xg, plan, nsamp=ns)), rows, 6, f"f32 apertif-like {name}")
    # every variant with a search epilogue (the asynchronous ones from index 13 on) fits this geometry
    names = dd.variant_names("f32")
    assert seen == sum(1 for i, n in enumerate(names) if i >= 13 and "_buf2" in n)


@pytest.mark.parametrize("ns", [1, 2, 7, 31, 32, 33, 100, 1239, 1240, 1241, 2500])
def test_f32_short_and_ragged(ns):
    dd = _dd()
    rng = np.random.default_rng(ns)
    nc, nd = 48, 37
    f = 1270.0 + (np.arange(nc) + 0.5) * 300.0 / nc
    dms = np.arange(nd) * 0.25
    delta = oracle.delay_table(f, 5e-5, dms)
    nin = ns + int(delta.max())
    x = rng.standard_normal((2, nc, nin)).astype(np.float32)
    plan = dd.Plan(f, 5e-5, dms)
    plan.set_detect_variant(13, "f32")
    assert plan.detect_variant("f32") == 13
    rows = oracle.forward_f32(x, delta, ns)
    for nw in (1, 6):
        _note(f"f32 short nsamp {ns} nwidth {nw}")
        got = _cpu(dd.detect(_to_gpu(x), plan, nsamp=ns, nwidth=nw))
        _check_f32(got, rows, nw, f"f32 ns{ns} nw{nw}", min_exact=0.9)


@pytest.mark.parametrize("ns", [1, 5, 31, 33, 991, 992, 993, 2049])
def test_u8_short_and_ragged(ns):
    dd = _dd()
    rng = np.random.default_rng(ns + 7)
    b = synth.config(2)[0]
    dms = b.dms()[:21]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, dms)
    nin = ns + int(delta.max())
    x = rng.integers(0, 256, (1, b.nchan, nin)).astype(np.uint8)
    plan = dd.Plan(b.freqs(), b.tsamp_s, dms)
    rows = oracle.forward_u8(x, delta, ns)
    for nw in (1, 6):
        _note(f"u8 short nsamp {ns} nwidth {nw}")
        got = _cpu(dd.detect(_to_gpu(x), plan, nsamp=ns, nwidth=nw))
        _check_exact(got, rows, nw, f"u8 ns{ns} nw{nw}")


def test_constant_input_is_degenerate():
    dd = _dd()
    b = synth.config(2)[0]
    dms = b.dms()[:8]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, dms)
    ns = 1500
    x = np.full((1, b.nchan, ns + int(delta.max())), 77, np.uint8)
    plan = dd.Plan(b.freqs(), b.tsamp_s, dms)
    got = _cpu(dd.detect(_to_gpu(x), plan, nsamp=ns))
    assert (got["snr"] == 0).all() and (got["width"] == 1).all() and (got["start"] == 0).all()
    assert (got["mean"] == 77 * b.nchan).all() and (got["std"] == 0).all()
    xf = np.full((1, 16, 3000), 0.5, np.float32)
    f = 1400.0 + np.arange(16) * 5.0
    pf = dd.Plan(f, 5e-5, [0.0, 1.0])
    got = _cpu(dd.detect(_to_gpu(xf), pf, nsamp=2000))
    assert (got["snr"] == 0).all() and (got["width"] == 1).all() and (got["start"] == 0).all()


def test_rows_search_matches_oracle_and_fused():
    dd = _dd()
    rng = np.random.default_rng(21)
    for n in (1, 40, 991, 992, 993, 5000):
        rows = rng.standard_normal((7, n)).astype(np.float32)
        rows[3, n // 2: n // 2 + min(n, 16)] += 4.0
        _note(f"rows f32 n {n}")
        got = _cpu(dd.detect_rows(torch.from_numpy(rows).cuda()))
        _check_f32(got, rows, 6, f"rows f32 n{n}", min_exact=0.85)
        ints = rng.integers(0, 8000, (5, n)).astype(np.int32)
        got = _cpu(dd.detect_rows(torch.from_numpy(ints).cuda(), nwidth=4))
        _check_exact(got, ints, 4, f"rows i32 n{n}")
    # the fused uint8 search equals the row search of the stored series
    b = synth.config(2)[0]
    dms = b.dms()[:50]
    plan = dd.Plan(b.freqs(), b.tsamp_s, dms)
    ns = 4000
    x = synth.noise(b, ns + plan.max_delay)[None]
    xg = _to_gpu(x)
    fused = _cpu(dd.detect(xg, plan, nsamp=ns))
    unfused = _cpu(dd.detect_rows(dd.dedisperse(xg, plan, nsamp=ns)))
    for k in fused:
        assert fused[k].shape == unfused[k].shape == (1, 50), k
        assert np.array_equal(fused[k], unfused[k]), k


def test_unfused_fallback_path():
    # delay spans too wide for every tiled variant: dedisperse into the
    # workspace with the direct kernel, then search the stored rows
    dd = _dd()
    nc, nd, ns = 16, 12, 3000
    f = 120.0 + np.arange(nc) * 2.0
    dms = np.arange(nd) * 40.0
    delta = oracle.delay_table(f, 1e-4, dms)
    plan = dd.Plan(f, 1e-4, dms)
    assert plan.detect_variant("f32") == -1 and plan.detect_variant("u8") == -1
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, nc, ns + int(delta.max()))).astype(np.float32)
    got = _cpu(dd.detect(_to_gpu(x), plan, nsamp=ns))
    _check_f32(got, oracle.forward_f32(x, delta, ns), 6, "fallback f32")
    xu = rng.integers(0, 256, (1, nc, ns + int(delta.max()))).astype(np.uint8)
    got = _cpu(dd.detect(_to_gpu(xu), plan, nsamp=ns))
    _check_exact(got, oracle.forward_u8(xu, delta, ns), 6, "fallback u8")


def test_config2_full_size_sampled():
    # the LOFAR-like workload at full size (2048 DMs x 200,000 samples, uint8),
    # checked on 48 DM trials spread over the range
    dd = _dd()
    b = synth.config(2)[0]
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    plan.autotune(1, b.nsamp, "u8")
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    x = synth.noise(b, b.nsamp + int(delta.max()))[None]
    _note(f"config2 full size, detect variant {plan.detect_variant('u8')}")
    got = _cpu(dd.detect(_to_gpu(x), plan, nsamp=b.nsamp))
    js = np.linspace(0, b.ndm - 1, 48).astype(int)
    rows = oracle.forward_u8(x, delta[js], b.nsamp)
    _check_exact({k: v[:, js] for k, v in got.items()}, rows, 6, "config2 sampled")


def test_config1_full_size_sampled():
    # the Apertif-like workload at full size (1024 channels, 2048 DMs, 20,000
    # samples, FP32, 8 injected pulses), checked on 32 DM trials and on the
    # pulses' own trials
    dd = _dd()
    b = synth.config(1)[0]
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    plan.autotune(1, b.nsamp, "f32")
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    x = synth.noise(b, b.nsamp + int(delta.max()))
    pulses = synth.pulses(b, int(delta.max()))
    for j, t0 in pulses:
        synth.inject(x, delta, j, t0, b.pulse_width, b.pulse_amp)
    _note(f"config1 full size, detect variant {plan.detect_variant('f32')}")
    got = _cpu(dd.detect(_to_gpu(x), plan, nsamp=b.nsamp))
    js = np.unique(np.concatenate([np.linspace(0, b.ndm - 1, 32).astype(int), [j for j, _ in pulses]]))
    rows = oracle.forward_f32(x[None], delta[js], b.nsamp)
    _check_f32({k: v[:, js] for k, v in got.items()}, rows, 6, "config1 sampled", min_exact=0.95)


def test_detect_errors():
    dd = _dd()
    b = synth.config(0)[0]
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    x = dd.empty_rows(1, b.nchan, b.nsamp + plan.max_delay, torch.float32, "cuda", zero=True)
    for nw in (0, 7):
        with pytest.raises(dd.DedispError):
            dd.detect(x, plan, nsamp=b.nsamp, nwidth=nw)
    with pytest.raises(dd.DedispError):
        dd.detect(x, plan, nsamp=b.nsamp, workspace=None, nwidth=-1)
    L = dd.lib()
    import ctypes
    o = torch.empty(b.ndm, dtype=torch.float64, device="cuda")
    wi = torch.empty(b.ndm, dtype=torch.int32, device="cuda")
    st = L.dedisp_detect(plan.handle, 1, b.nsamp, ctypes.c_void_p(x.data_ptr()), 0, x.stride(1), None, 6,
                         ctypes.c_void_p(o.data_ptr()), ctypes.c_void_p(wi.data_ptr()),
                         ctypes.c_void_p(wi.data_ptr()), None, None, ctypes.c_void_p(o.data_ptr()), 8, None)
    assert st == 8  # workspace too small


def test_detect_autotune_and_forced_paths():
    # the tuner times every fused variant and the unfused path and keeps one;
    # every path gives the same uint8 result
    dd = _dd()
    b = synth.config(2)[0]
    dms = b.dms()[:64]
    plan = dd.Plan(b.freqs(), b.tsamp_s, dms)
    ns = 6000
    x = synth.noise(b, ns + plan.max_delay)[None]
    xg = _to_gpu(x)
    times = plan.autotune_detect(1, ns, "u8")
    _note(f"detect autotune: {times}")
    assert "unfused" in times and len(times) >= 9
    best = min(times, key=times.get)
    chosen = plan.detect_variant("u8")
    assert (best == "unfused" and chosen == -1) or dd.variant_names("u8")[chosen] == best
    ref = _cpu(dd.detect(xg, plan, nsamp=ns))
    _check_exact(ref, oracle.forward_u8(x, oracle.delay_table(b.freqs(), b.tsamp_s, dms), ns), 6, "tuned")
    for v in (-1, 12, 16, 20):
        plan.set_detect_variant(v, "u8")
        assert plan.detect_variant("u8") == v
        got = _cpu(dd.detect(xg, plan, nsamp=ns))
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (v, k)
    with pytest.raises(dd.DedispError):
        plan.set_detect_variant(0, "u8")  # one-copy variant: no search epilogue
    plan.set_detect_variant(-2, "u8")
    assert plan.detect_variant("u8") >= 0
