"""GPU checks of the batched (persistent, graph-captured) path: equal bit for
bit to the per-beam launch loop, equal to the oracle, and deterministic
across graph replays."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def _dd():
    import paper_1601_01165_amd as dd

    return dd


def _note(msg):
    print(msg, flush=True)


def _small_batch(nbeam=7, seed=31):
    """Uneven beams in the band of the batched workload, scaled down."""
    rng = np.random.default_rng(seed)
    beams = []
    for i in range(nbeam):
        nc = int(rng.choice([64, 128, 256, 300]))
        nd = int(rng.integers(20, 200))
        ns = int(rng.integers(500, 3000))
        beams.append(synth.Beam(nc, 1270.0, 1570.0, 50e-6, ns, nd, 0.25, "f32", seed * 100 + i, npulse=2))
    return beams


def _setup(beams, weighted=False):
    dd = _dd()
    plans, xs, outs, ref_in, deltas, ws = [], [], [], [], [], []
    for b in beams:
        delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
        nin = b.nsamp + int(delta.max())
        x = synth.noise(b, nin)
        for j, t0 in synth.pulses(b, int(delta.max())):
            synth.inject(x, delta, j, t0, b.pulse_width, b.pulse_amp)
        xg = dd.empty_rows(1, b.nchan, nin, torch.float32, "cuda")
        xg.copy_(torch.from_numpy(x)[None])
        plans.append(dd.Plan(b.freqs(), b.tsamp_s, b.dms()))
        xs.append(xg)
        outs.append(dd.empty_rows(1, b.ndm, b.nsamp, torch.float32, "cuda", zero=True))
        ref_in.append(x)
        deltas.append(delta)
        if weighted:
            ws.append(torch.from_numpy(np.random.default_rng(b.seed).uniform(0.5, 1.5, b.nchan).astype(np.float32))
                      .cuda())
    return plans, xs, outs, ref_in, deltas, (ws if weighted else None)


@pytest.mark.parametrize("weighted", [False, True])
def test_batched_matches_per_beam_and_oracle(weighted):
    dd = _dd()
    beams = _small_batch()
    plans, xs, outs, ref_in, deltas, ws = _setup(beams, weighted)
    batch = dd.Batch(plans, xs, outs, weights=ws)
    _note(f"batched execute weighted={weighted}")
    batch.execute()
    torch.cuda.synchronize()
    got_b = [o.cpu().numpy().copy() for o in outs]
    for o in outs:
        o.zero_()
    _note("per-beam loop")
    batch.execute_per_beam()
    torch.cuda.synchronize()
    got_p = [o.cpu().numpy().copy() for o in outs]
    for i, b in enumerate(beams):
        assert np.array_equal(got_b[i], got_p[i]), f"beam {i}: batched != per-beam"
        w = None if ws is None else ws[i].cpu().numpy()
        ref = oracle.forward_f32(ref_in[i], deltas[i], b.nsamp, w)
        assert np.array_equal(got_b[i], ref), f"beam {i}: batched != oracle"


def test_graph_replay_deterministic():
    dd = _dd()
    beams = _small_batch(5, seed=37)
    plans, xs, outs, ref_in, deltas, _ = _setup(beams)
    batch = dd.Batch(plans, xs, outs)
    results = []
    for r in range(3):
        _note(f"replay {r}")
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        batch.execute()
        torch.cuda.synchronize()
        results.append([o.cpu().numpy().copy() for o in outs])
    for r in range(1, 3):
        for i in range(len(beams)):
            assert np.array_equal(results[0][i], results[r][i])
    for i, b in enumerate(beams):
        assert np.array_equal(results[0][i], oracle.forward_f32(ref_in[i], deltas[i], b.nsamp))


def test_batched_tuned_matches():
    dd = _dd()
    beams = _small_batch(4, seed=41)
    plans, xs, outs, ref_in, deltas, _ = _setup(beams)
    batch = dd.Batch(plans, xs, outs, tune=True)
    _note("tuned batch")
    for o in outs:
        o.zero_()
    batch.execute()
    torch.cuda.synchronize()
    for i, b in enumerate(beams):
        assert np.array_equal(outs[i].cpu().numpy(), oracle.forward_f32(ref_in[i], deltas[i], b.nsamp))


def test_autotune_single_plan_and_cache(tmp_path):
    dd = _dd()
    b = synth.config(0)[0]
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    cache = str(tmp_path / "tune.json")
    _note("autotune f32")
    times = plan.autotune(1, b.nsamp, "f32", cache)
    assert "direct" in times and any(v > 0 for v in times.values())
    chosen = plan.variant("f32")
    txt = open(cache).read()
    assert "variant" in txt
    plan2 = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    plan2.autotune(1, b.nsamp, "f32", cache)  # cache hit
    assert plan2.variant("f32") == chosen
    # the tuned plan still matches the oracle
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    x = synth.noise(b, nin)
    xg = dd.empty_rows(1, b.nchan, nin, torch.float32, "cuda")
    xg.copy_(torch.from_numpy(x)[None])
    out = dd.dedisperse(xg, plan2, nsamp=b.nsamp)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.forward_f32(x, delta, b.nsamp))


@pytest.mark.parametrize("weighted", [False, True])
def test_batched_every_variant(weighted):
    """The persistent kernel of every FP32 variant that fits the beams (the
    pipelined two-window ones included) against the oracle; a variant that
    does not fit is refused and leaves the batch runnable."""
    dd = _dd()
    beams = _small_batch(5, seed=43)
    plans, xs, outs, ref_in, deltas, ws = _setup(beams, weighted)
    batch = dd.Batch(plans, xs, outs, weights=ws)
    names = dd.variant_names("f32")
    ran = 0
    for v in range(len(names)):
        try:
            batch.set_variant(v)
        except dd.DedispError:
            _note(f"variant {v} {names[v]} does not fit")
            continue
        assert batch.variant == v
        _note(f"batched variant {v} {names[v]} weighted={weighted}")
        for o in outs:
            o.fill_(float("nan"))
        batch.execute()
        torch.cuda.synchronize()
        for i, b in enumerate(beams):
            w = None if ws is None else ws[i].cpu().numpy()
            ref = oracle.forward_f32(ref_in[i], deltas[i], b.nsamp, w)
            assert np.array_equal(outs[i].cpu().numpy(), ref), (v, i)
        ran += 1
    assert ran >= len(names) // 2
    with pytest.raises(dd.DedispError):
        batch.set_variant(len(names))
    batch.execute()
    torch.cuda.synchronize()


def test_config3_full_size_sampled():
    """The batched workload at full size (256 uneven beams, 20.7 GB in, 33.9 GB
    out) in the tuned persistent launch the benchmark times, checked against
    the oracle on 4,000 sampled outputs of each of 10 beams (the beams with
    the most channels and the most DM trials among them), bit for bit."""
    dd = _dd()
    beams = synth.config(3)
    plans, xs, outs = [], [], []
    for i, b in enumerate(beams):
        p = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
        x = dd.empty_rows(1, b.nchan, b.nsamp + p.max_delay, torch.float32, "cuda")
        g = torch.Generator(device="cuda")
        g.manual_seed(b.seed)
        x.copy_(torch.randn(x.shape, generator=g, device="cuda"))
        plans.append(p)
        xs.append(x)
        outs.append(dd.empty_rows(1, b.ndm, b.nsamp, torch.float32, "cuda"))
        if i % 64 == 63:
            _note(f"config3: {i + 1} beams prepared")
    batch = dd.Batch(plans, xs, outs, tune=True)
    _note(f"config3: tuned variant {dd.variant_names('f32')[batch.variant]}")
    for o in outs:
        o.fill_(float("nan"))
    batch.execute()
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    pick = set(rng.choice(len(beams), 8, replace=False).tolist())
    pick.add(max(range(len(beams)), key=lambda i: beams[i].nchan * beams[i].ndm))
    pick.add(max(range(len(beams)), key=lambda i: beams[i].ndm))
    for i in sorted(pick):
        b = beams[i]
        delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
        x = np.ascontiguousarray(xs[i].cpu().numpy())
        pd = rng.integers(0, b.ndm, 4000)
        ps = rng.integers(0, b.nsamp, 4000)
        pd[:2] = [0, b.ndm - 1]
        ps[:2] = [0, b.nsamp - 1]
        ref, _ = oracle.forward_points(x, delta, np.zeros(4000, np.int32), pd, ps)
        got = outs[i][0].cpu().numpy()[pd, ps]
        _note(f"config3 beam {i}: {b.nchan} ch, {b.ndm} DMs, {b.nsamp} samples")
        assert np.array_equal(got, ref), f"beam {i}"


def test_batched_tune_cache_hit(tmp_path):
    """The batch's tuning is stored in the cache file and a second batch of
    the same shapes takes it from there (no search), with the same variant and
    results still equal to the oracle."""
    dd = _dd()
    cache = str(tmp_path / "batch_tune.json")
    beams = _small_batch(4, seed=47)
    plans, xs, outs, ref_in, deltas, _ = _setup(beams)
    _note("tuned batch, cold cache")
    b1 = dd.Batch(plans, xs, outs, tune=True, tune_cache=cache)
    assert not b1.cache_hit
    v1 = b1.variant
    assert "|batch|f32|w0|n4|" in open(cache).read()
    _note("tuned batch, warm cache")
    b2 = dd.Batch(plans, xs, outs, tune=True, tune_cache=cache)
    assert b2.cache_hit and b2.variant == v1
    for o in outs:
        o.fill_(float("nan"))
    b2.execute()
    torch.cuda.synchronize()
    for i, b in enumerate(beams):
        assert np.array_equal(outs[i].cpu().numpy(), oracle.forward_f32(ref_in[i], deltas[i], b.nsamp)), i
    # other shapes miss the cache
    beams3 = _small_batch(3, seed=53)
    plans3, xs3, outs3, _, _, _ = _setup(beams3)
    assert not dd.Batch(plans3, xs3, outs3, tune=True, tune_cache=cache).cache_hit


def test_batched_refuses_uint8_and_bad_beams():
    """uint8 batches are refused by the C-ABI with the dtype status; buffers
    that do not match their plan are refused before the library is called."""
    dd = _dd()
    from paper_1601_01165_amd import _clib
    import ctypes

    beams = _small_batch(2, seed=59)
    plans, xs, outs, _, _, _ = _setup(beams)
    L = dd.lib()
    n = 2
    arr = lambda typ, vals: (typ * n)(*vals)  # noqa: E731
    h = ctypes.c_void_p()
    st = L.dedisp_batch_create(ctypes.byref(h), n, arr(ctypes.c_void_p, [p.handle.value for p in plans]),
                               arr(ctypes.c_int32, [b.nsamp for b in beams]),
                               arr(ctypes.c_void_p, [x.data_ptr() for x in xs]), _clib.U8,
                               arr(ctypes.c_int64, [x.stride(1) for x in xs]), None,
                               arr(ctypes.c_void_p, [o.data_ptr() for o in outs]),
                               arr(ctypes.c_int64, [o.stride(1) for o in outs]), 0, None)
    assert st == _clib.E_DTYPE
    with pytest.raises(ValueError, match="DM rows"):
        dd.Batch(plans, xs, outs[::-1])
    with pytest.raises(ValueError, match="GPU"):
        dd.Batch(plans, xs, outs, weights=[torch.ones(p.nchan) for p in plans])
