"""Streaming: consecutive chunks of one long observation, each chunk's input
an in-place view of the long rows that starts at the chunk's first sample and
carries the max-delay halo after it (the input length of Section 2.1: the
samples one chunk of output needs, delays included; Section 5.1's real-time
use processes one second after the other).  Every chunk's output is compared
with the oracle evaluated on the long input at the same absolute samples."""
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


def _long_input(b, nchunk, halo, seed):
    dd = _dd()
    n = nchunk * b.nsamp + halo
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((b.nchan, n), dtype=np.float32)
    xg = dd.empty_rows(1, b.nchan, n, torch.float32, "cuda")
    xg.copy_(torch.from_numpy(x)[None])
    return x, xg


def test_streamed_chunks_small_whole_outputs():
    """Three chunks of two beams through the batched launch and through
    dedisperse on the chunk views; every output element against the oracle."""
    dd = _dd()
    b = synth.Beam(256, 1270.0, 1570.0, 50e-6, 3000, 200, 0.25, "f32", 71)
    nchunk = 3
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    halo = int(delta.max())
    beams = [_long_input(b, nchunk, halo, s) for s in (1, 2)]
    outs = [dd.empty_rows(1, b.ndm, nchunk * b.nsamp, torch.float32, "cuda", zero=True) for _ in beams]
    batches = []
    for k in range(nchunk):
        xin = [xg[:, :, k * b.nsamp:(k + 1) * b.nsamp + halo] for _, xg in beams]
        oin = [o[:, :, k * b.nsamp:(k + 1) * b.nsamp] for o in outs]
        batches.append(dd.Batch([plan] * len(beams), xin, oin))
    for k, bt in enumerate(batches):
        _note(f"chunk {k}: batched")
        bt.execute()
    torch.cuda.synchronize()
    for (x, xg), o in zip(beams, outs):
        whole = oracle.forward_f32(x, delta, nchunk * b.nsamp)[0]
        assert np.array_equal(o[0].cpu().numpy(), whole)
        for k in range(nchunk):
            _note(f"chunk {k}: dedisperse on the view")
            view = xg[:, :, k * b.nsamp:(k + 1) * b.nsamp + halo]
            got = dd.dedisperse(view, plan, nsamp=b.nsamp)
            torch.cuda.synchronize()
            ref = oracle.forward_f32(np.ascontiguousarray(x[:, k * b.nsamp:(k + 1) * b.nsamp + halo]), delta,
                                     b.nsamp)[0]
            assert np.array_equal(got[0].cpu().numpy(), ref), k
            assert np.array_equal(ref, whole[:, k * b.nsamp:(k + 1) * b.nsamp])


def test_streamed_chunks_apertif_full_size_sampled():
    """The Apertif-like beam (1024 channels, 2048 DM trials, 1 s chunks of
    20,000 samples with the 9,093-sample halo), three consecutive chunks in
    place through the batched launch: 5,000 sampled
    outputs and two whole rows per chunk against the oracle on the long input."""
    dd = _dd()
    b = synth.config(1)[0]
    nchunk = 3
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    halo = int(delta.max())
    _note("apertif stream: generating the long input")
    x, xg = _long_input(b, nchunk, halo, 73)
    out = dd.empty_rows(1, b.ndm, nchunk * b.nsamp, torch.float32, "cuda", zero=True)
    bt = [dd.Batch([plan], [xg[:, :, k * b.nsamp:(k + 1) * b.nsamp + halo]],
                   [out[:, :, k * b.nsamp:(k + 1) * b.nsamp]]) for k in range(nchunk)]
    for k in range(nchunk):
        _note(f"apertif stream chunk {k}")
        bt[k].execute()
    torch.cuda.synchronize()
    o = out[0].cpu().numpy()
    rng = np.random.default_rng(74)
    for k in range(nchunk):
        pd = rng.integers(0, b.ndm, 5000).astype(np.int32)
        ps = (k * b.nsamp + rng.integers(0, b.nsamp, 5000)).astype(np.int32)
        pd[:4] = [0, b.ndm - 1, 0, b.ndm - 1]
        ps[:4] = [k * b.nsamp, k * b.nsamp, (k + 1) * b.nsamp - 1, (k + 1) * b.nsamp - 1]
        ref, _ = oracle.forward_points(x[None], delta, np.zeros(pd.size, np.int32), pd, ps)
        assert np.array_equal(o[pd, ps], ref), k
        rows = [int(rng.integers(0, b.ndm)), b.ndm - 1]
        full = oracle.forward_f32(np.ascontiguousarray(x[:, k * b.nsamp:(k + 1) * b.nsamp + halo]), delta[rows],
                                  b.nsamp)[0]
        assert np.array_equal(o[rows, k * b.nsamp:(k + 1) * b.nsamp], full), k
