"""The paper's tuning experiments, repeated on MI355X with this library.

python -m paper_1601_01165_amd.experiments [--quick]

Prints one JSON object per experiment:

* ``tuned_vs_generic`` (Section 5, "generically tuned": one-dimensional
  work-groups, one DM per work-item, no data reuse): for the Apertif-like and
  LOFAR-like set-ups and a range of DM counts (the paper uses 2 to 4,096), the
  auto-tuned time and the direct kernel's time, and their ratio.
* ``perfect_reuse`` (Section 4.3): the same set-ups with every DM trial set to
  zero, so every trial reads the same input; tuned time against the real DM
  list.
* ``histogram`` (Section 4.2): the time of every compiled variant on the
  Apertif-like set-up with 2,048 DMs (the distribution of the tuning space).
* ``scaling``: throughput against the number of DMs (the shape of the paper's
  performance-versus-instance-size figures).
* ``realtime_beams`` (Section 5.1): Apertif-like beams with 2,000 DMs
  dedispersed per second of compute, i.e. beams one GPU keeps up with in real
  time (the paper: 9 per HD7970).
* ``streaming``: the same as a stream of consecutive 1 s chunks with a
  max-delay halo, each chunk one graph replay, checked against one long run.
* ``detect``: dedispersion followed by the single-pulse search (boxcar S/N,
  widths 1..32) on the Apertif-like (2,000 DMs) and LOFAR-like (2,048 DMs)
  set-ups: the tuned search path against the unfused one, and the beams one
  GPU dedisperses and searches in real time.

All inputs are synthetic (seeded noise); only timings are reported.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import Batch, Plan, dedisperse, detect, empty_rows


def _setup(name):
    # centre frequencies of equal sub-bands, as in the workloads of the tests
    if name == "apertif":
        nc, lo, hi, ts, ns, step, dtype = 1024, 1270.0, 1570.0, 50e-6, 20000, 0.25, torch.float32
    else:
        nc, lo, hi, ts, ns, step, dtype = 32, 134.875, 141.125, 5e-6, 200000, 0.01, torch.uint8
    f = lo + (np.arange(nc) + 0.5) * (hi - lo) / nc
    return f, ts, ns, step, dtype


def _input(nc, nin, dtype, seed):
    x = empty_rows(1, nc, nin, dtype, "cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    v = torch.randn(x.shape, generator=g, device="cuda")
    if dtype == torch.uint8:
        x.copy_(torch.clamp(torch.round(128.0 + 16.0 * v), 0, 255).to(torch.uint8))
    else:
        x.copy_(v)
    return x


def _time(fn, reps=5):
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def tuned_vs_generic(name, ndms, perfect=False):
    f, ts, ns, step, dtype = _setup(name)
    dt = "u8" if dtype == torch.uint8 else "f32"
    rows = []
    for nd in ndms:
        dms = np.zeros(nd) if perfect else np.arange(nd) * step
        p = Plan(f, ts, dms)
        nin = ns + p.max_delay
        x = _input(len(f), nin, dtype, 7)
        out = empty_rows(1, nd, ns, torch.int32 if dt == "u8" else torch.float32, "cuda")
        times = p.autotune(1, ns, dt)
        tuned = min(v for v in times.values() if v > 0)
        best = min((v, k) for k, v in times.items() if v > 0)[1]
        p.set_variant(-1, dt)
        generic = _time(lambda: dedisperse(x, p, nsamp=ns, out=out))
        rows.append({"ndm": nd, "tuned_ms": tuned, "tuned_variant": best, "generic_ms": generic,
                     "speedup": generic / tuned,
                     "gflops_tuned": len(f) * nd * ns / (tuned * 1e-3) / 1e9})
        del x, out, p
    return rows


def histogram(name="apertif", nd=2048):
    f, ts, ns, step, dtype = _setup(name)
    p = Plan(f, ts, np.arange(nd) * step)
    _input(len(f), ns + p.max_delay, dtype, 7)
    times = p.autotune(1, ns, "u8" if dtype == torch.uint8 else "f32")
    return {k: v for k, v in sorted(times.items(), key=lambda kv: kv[1])}


def realtime_beams(nbeams=64, nd=2000):
    f, ts, ns, step, dtype = _setup("apertif")
    plans, xs, outs = [], [], []
    for b in range(nbeams):
        p = Plan(f, ts, np.arange(nd) * step)
        plans.append(p)
        xs.append(_input(len(f), ns + p.max_delay, dtype, 100 + b))
        outs.append(empty_rows(1, nd, ns, torch.float32, "cuda"))
    batch = Batch(plans, xs, outs, tune=True)
    ms = _time(batch.execute, reps=3)
    seconds_of_data = nbeams * ns * ts
    return {"beams": nbeams, "ndm": nd, "ms": ms, "beams_realtime": seconds_of_data / (ms * 1e-3),
            "paper_hd7970_beams": 9}


def streaming(nbeams=16, nchunks=4, nd=2000):
    """Consecutive 1 s chunks of Apertif-like beams with a max-delay halo
    (Section 5.1's real-time set-up, Section 2's input length): each beam's
    samples sit in one long row per channel; chunk k reads samples
    [k*S, (k+1)*S + max_delay) in place, so consecutive chunks overlap by the
    halo and nothing is copied.  One graph-captured batch per chunk offset is
    replayed in order.  Checks that the chunked outputs equal one long run,
    then reports the beams kept in real time."""
    f, ts, ns, step, dtype = _setup("apertif")
    plans, xs, outs = [], [], []
    for b in range(nbeams):
        p = Plan(f, ts, np.arange(nd) * step)
        plans.append(p)
        xs.append(_input(len(f), nchunks * ns + p.max_delay, dtype, 300 + b))
        outs.append(empty_rows(1, nd, nchunks * ns, torch.float32, "cuda"))
    batches = []
    for k in range(nchunks):
        xin = [x[:, :, k * ns: (k + 1) * ns + p.max_delay] for x, p in zip(xs, plans)]
        oin = [o[:, :, k * ns: (k + 1) * ns] for o in outs]
        batches.append(Batch(plans, xin, oin, tune=(k == 0)))
        if k > 0:
            batches[k].set_variant(batches[0].variant)

    def run():
        for bt in batches:
            bt.execute()
    ms = _time(run, reps=3)
    # the chunked result equals one long run of each beam
    ok = True
    for x, p, o in zip(xs[:2], plans[:2], outs[:2]):
        whole = dedisperse(x, p, nsamp=nchunks * ns)
        ok = ok and bool(torch.equal(whole, o))
    seconds_of_data = nbeams * nchunks * ns * ts
    return {"beams": nbeams, "chunks": nchunks, "chunk_s": ns * ts, "ndm": nd, "halo_samples": plans[0].max_delay,
            "ms": ms, "chunked_equals_whole": ok, "beams_realtime": seconds_of_data / (ms * 1e-3)}


def detect_realtime(name, nd):
    f, ts, ns, step, dtype = _setup(name)
    dt = "u8" if dtype == torch.uint8 else "f32"
    p = Plan(f, ts, np.arange(nd) * step)
    x = _input(len(f), ns + p.max_delay, dtype, 11)
    p.autotune(1, ns, dt)
    paths = p.autotune_detect(1, ns, dt)
    chosen = p.detect_variant(dt)
    ws = torch.empty(nd * (ns + 4) * 4 + (1 << 26), dtype=torch.uint8, device="cuda")
    tuned = _time(lambda: detect(x, p, nsamp=ns, workspace=ws))
    p.set_detect_variant(-1, dt)
    unfused = _time(lambda: detect(x, p, nsamp=ns, workspace=ws))
    fused = {k: v for k, v in paths.items() if k != "unfused"}
    return {"setup": name, "ndm": nd, "samples": ns, "tuned_ms": tuned, "unfused_ms": unfused,
            "best_fused_ms": min(fused.values()) if fused else None,
            "chosen": "unfused" if chosen < 0 else min(fused, key=fused.get),
            "beams_realtime": ns * ts / (tuned * 1e-3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args()
    ndms = [2, 16, 128, 512, 2048] if args.quick else [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096]
    t0 = time.time()
    for name in ("apertif", "lofar"):
        print(json.dumps({"experiment": "tuned_vs_generic", "setup": name, "rows": tuned_vs_generic(name, ndms)}),
              flush=True)
        print(json.dumps({"experiment": "perfect_reuse", "setup": name,
                          "rows": tuned_vs_generic(name, [ndms[-1]], perfect=True)}), flush=True)
    print(json.dumps({"experiment": "histogram", "setup": "apertif", "ndm": 2048, "ms": histogram()}), flush=True)
    print(json.dumps({"experiment": "realtime_beams", **realtime_beams(16 if args.quick else 64)}), flush=True)
    print(json.dumps({"experiment": "streaming", **streaming(8 if args.quick else 16)}), flush=True)
    for name, nd in (("apertif", 2000), ("lofar", 2048)):
        print(json.dumps({"experiment": "detect", **detect_realtime(name, nd)}), flush=True)
    print(f"experiments done in {time.time() - t0:.1f} s", file=sys.stderr)


if __name__ == "__main__":
    main()
