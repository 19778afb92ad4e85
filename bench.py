#!/usr/bin/env python3
"""Benchmark of brute-force dedispersion on one MI355X.

Default workload: 256 uneven beams (per beam, seeded: 256/512/1024/1536
channels over 1270-1570 MHz, 512-4096 DM trials in steps of 0.25, 8000-20000
output samples, 50 us sampling, FP32 noise with two injected pulses), run as
one persistent, graph-captured launch with the tile shape chosen by the
autotuner, and compared with a loop of per-beam launches (each beam's plan
tuned on its own).  One step = one pass over all beams; inputs are resident
in HBM before the timed region.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DM-trial·samples/s (GB/s and % of HBM roofline), batched vs plain"
HBM_PEAK = 8.0e12            # B/s, MI355X HBM3E
ADD_PEAK = 157.3e12 / 2      # FP32 adds/s: 157.3 TFLOP/s counts an FMA as 2 flops; an add is 1
T0 = time.time()


def log(msg):
    print(f"[bench {time.time() - T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched",
                    choices=["batched", "apertif", "lofar", "diff", "detect_apertif", "detect_lofar", "copy"],
                    help="copy: a plain 1 GiB device copy, the reference for HBM byte counters")
    ap.add_argument("--no-tune", action="store_true", help="use default variants (no autotuning)")
    ap.add_argument("--variant", type=int, default=None, help="force a kernel variant (no autotuning)")
    ap.add_argument("--queues", type=int, default=0, help="batched: force 1 or 8 work queues")
    ap.add_argument("--weights", action="store_true",
                    help="apertif: per-channel weights (all ones), i.e. the fused multiply-add path")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-beam loop")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-tuned", action="store_true", help="skip the tuned multi-core CPU comparator")
    ap.add_argument("--cpu-tuned-seconds", type=float, default=5.0, help="target time of the tuned CPU run")
    ap.add_argument("--beams", type=int, default=0, help="use only the first N beams (debugging)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="batched workload: skip the LOFAR-like and differentiable workloads timed after it")
    ap.add_argument("--no-cold", action="store_true",
                    help="skip the cold-cache runs (single-beam workloads: each run after a 512 MB scratch write)")
    return ap.parse_args()


def fill_noise(t, seed):
    import torch

    g = torch.Generator(device=t.device)
    g.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    t.copy_(torch.randn(t.shape, generator=g, device=t.device, dtype=t.dtype))


def inject_device(x, delta_row, t0, width, amp):
    """x[c][t0 + delta[c] + k] += amp for k < width (x: [C][nin] on the GPU)."""
    import torch

    c = torch.arange(x.shape[0], device=x.device)
    d = torch.from_numpy(delta_row.astype(np.int64)).to(x.device)
    for k in range(width):
        x[c, t0 + d + k] += amp


def time_steps(fn, steps, warmup, stream_sync):
    import torch

    for _ in range(warmup):
        fn()
    stream_sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    per = []
    t_start = time.perf_counter()
    e0.record()
    for _ in range(steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        per.append((a, b))
    e1.record()
    stream_sync()
    wall = time.perf_counter() - t_start
    total_ms = e0.elapsed_time(e1)
    launch_ms = [a.elapsed_time(b) for a, b in per]
    return total_ms / steps, launch_ms, wall


def time_cold(fn, runs, stream_sync):
    """Per-run times (ms, HIP events on the launch stream) with every run
    preceded by a 512 MB scratch write, more than the 256 MB MALL and the L2s
    hold, so the run's inputs come from HBM.  The write is outside the timed
    region."""
    import torch

    scratch = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    per = []
    for i in range(runs):
        scratch.fill_(i & 0xFF)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        per.append((a, b))
    stream_sync()
    del scratch
    return [a.elapsed_time(b) for a, b in per]


def cpu_model():
    """The host CPU's model name and logical CPU count, as the OS reports them."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    name = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": name, "logical_cpus": os.cpu_count()}


def cpu_baseline(beam, target_s, search=False):
    """Time the plain oracle on a bounded sample of one beam: all channels and
    samples, a prefix of the DM trials sized for ~target_s seconds (with
    search: each dedispersed series also goes through the oracle's boxcar
    search)."""
    import oracle
    import synth

    oracle.build()
    delta = oracle.delay_table(beam.freqs(), beam.tsamp_s, beam.dms())
    nin = beam.nsamp + int(delta.max())
    x = synth.noise(beam, nin)
    fwd0 = oracle.forward_u8 if beam.dtype == "u8" else oracle.forward_f32

    def fwd(x, d, n):
        y = fwd0(x, d, n)
        if search:
            oracle.detect(y, 6)
        return y
    # calibrate on two DM trials per thread (rows are the unit of parallelism)
    nth = max(1, oracle.num_threads())
    ncal = min(beam.ndm, 2 * nth)
    fwd(x, delta[:nth], beam.nsamp)  # warm threads and caches
    t = time.perf_counter()
    fwd(x, delta[:ncal], beam.nsamp)
    dtc = time.perf_counter() - t
    nd = int(ncal * target_s / max(dtc, 1e-6))
    nd = max(nth, nd - nd % nth)
    reps = 1
    if nd > beam.ndm:  # the whole beam is cheaper than the target: repeat it
        reps = max(1, int(round(nd / beam.ndm)))
        nd = beam.ndm
    t = time.perf_counter()
    for _ in range(reps):
        fwd(x, delta[:nd], beam.nsamp)
    el = time.perf_counter() - t
    what = f"first {nd} of {beam.ndm} DM trials" if nd < beam.ndm else f"all {nd} DM trials, {reps} time(s)"
    arith = "uint8 in, int32 sums" if beam.dtype == "u8" else "FP32"
    if search:
        arith += ", then the FP64 boxcar search of widths 1..32"
    return {
        "value": reps * nd * beam.nsamp / el,
        "unit": "DM-trial·samples/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "host": cpu_model(),
        "sample": f"one beam: {beam.nchan} channels x {beam.nsamp} samples, {what} "
                  f"(Algorithm 1 order, {arith}), {el:.1f} s",
        "seconds": el,
    }


def cpu_baseline_subset(beams, target_s, nsub=16, seed=1704):
    """Time the plain oracle on a seeded subset of the batched workload's
    beams: nsub beams drawn without replacement; of each, all channels and
    samples and a prefix of its DM trials sized so that each beam gets an
    equal share of what is left of target_s (calibrated on two DM trials per
    thread of the first beam and scaled by channels x samples; a beam with
    fewer DM trials than its share leaves the rest to the later ones).  The rate is the subset's
    DM-trial.samples over the summed time."""
    import oracle
    import synth

    oracle.build()
    idx = sorted(np.random.default_rng(seed).choice(len(beams), size=min(nsub, len(beams)), replace=False).tolist())
    nth = max(1, oracle.num_threads())
    per_row = None
    total_rows_samples = 0
    total_s = 0.0
    parts = []
    for n, i in enumerate(idx):
        beam = beams[i]
        delta = oracle.delay_table(beam.freqs(), beam.tsamp_s, beam.dms())
        x = synth.noise(beam, beam.nsamp + int(delta.max()))
        if per_row is None:
            ncal = min(beam.ndm, 2 * nth)
            oracle.forward_f32(x, delta[:nth], beam.nsamp)  # warm threads and caches
            t = time.perf_counter()
            oracle.forward_f32(x, delta[:ncal], beam.nsamp)
            # seconds per DM trial per (channel x sample), all threads busy
            per_row = (time.perf_counter() - t) / ncal / (beam.nchan * beam.nsamp)
        # this beam's share of what is left of the budget
        nd = int((target_s - total_s) / (len(idx) - n) / (per_row * beam.nchan * beam.nsamp))
        nd = min(beam.ndm, max(nth, nd - nd % nth))
        t = time.perf_counter()
        oracle.forward_f32(x, delta[:nd], beam.nsamp)
        el = time.perf_counter() - t
        total_rows_samples += nd * beam.nsamp
        total_s += el
        parts.append(f"{beam.nchan}ch/{nd} of {beam.ndm} DMs/{beam.nsamp} samples")
        if n % 4 == 3:
            log(f"  cpu baseline: {n + 1} of {len(idx)} beams")
    return {
        "value": total_rows_samples / total_s,
        "unit": "DM-trial·samples/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "host": cpu_model(),
        "sample": f"{len(idx)} beams of the {len(beams)} drawn with seed {seed} (beam indices {idx}); of each, all "
                  f"channels and samples and the first DM trials: " + ", ".join(parts) +
                  f" (Algorithm 1 order, FP32), {total_s:.1f} s",
        "seconds": total_s,
    }


def cpu_tuned(beam, target_s):
    """Time the tuned multi-core CPU implementation (the paper's CPU
    comparison, Section 5: tiles of DMs x samples, SIMD over samples, threads
    over tiles) on one whole beam: its tile shape is tuned first on a 64-DM
    slice, then the beam is repeated until ~target_s seconds have run.  The
    output of the first repeat is checked against the oracle on sampled DM
    trials."""
    import oracle
    import synth
    from paper_1601_01165_amd import cpu

    cpu.build_if_missing()
    delta = oracle.delay_table(beam.freqs(), beam.tsamp_s, beam.dms())
    nin = beam.nsamp + int(delta.max())
    x = synth.noise(beam, nin)[None]
    times, best = cpu.autotune(x, delta[:64], beam.nsamp, reps=3)
    t = time.perf_counter()
    out = cpu.forward(x, delta, beam.nsamp, cfg=best)
    one = time.perf_counter() - t
    reps = max(1, int(round(target_s / max(one, 1e-6))))
    t = time.perf_counter()
    for _ in range(reps):
        cpu.forward(x, delta, beam.nsamp, cfg=best, out=out)
    el = time.perf_counter() - t
    rows = np.linspace(0, beam.ndm - 1, 4).astype(int)
    fwd = oracle.forward_u8 if beam.dtype == "u8" else oracle.forward_f32
    ok = bool(np.array_equal(out[0, rows], fwd(x, delta[rows], beam.nsamp)[0]))
    dt, ds = cpu.configs()[best]
    return {
        "value": reps * beam.ndm * beam.nsamp / el,
        "unit": "DM-trial·samples/s",
        "cores": cpu.num_threads(),
        "kind": "tuned-cpu",
        "isa": cpu.isa(),
        "tile": {"dms": dt, "samples": ds},
        "matches_oracle": ok,
        "sample": f"one beam: {beam.nchan} channels x {beam.nsamp} samples x {beam.ndm} DM trials, "
                  f"{reps} time(s), {el:.1f} s",
        "seconds": el,
    }


def kernel_sources_hash():
    """Hash of the kernel sources: stored byte counters apply only to the kernels they were taken on."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1601_01165_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        # the sources, including the generator of the inner steps (its output is not tracked)
        if f.endswith((".hip", ".h", ".py")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload, variant):
    """HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE +
    WRITE_SIZE, scaled by the same counters of a plain copy of known size),
    from the summary committed under profiles/; None if there is none for
    this workload and variant or the kernels changed since."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    want = kernel_sources_hash()
    for ln in open(path):
        if not ln.startswith("traffic "):
            continue
        kv = dict(tok.split("=", 1) for tok in ln.split()[1:])
        # variant names are stored with spaces as underscores (the line is whitespace-separated)
        if kv.get("workload") == workload and kv.get("variant") == variant.replace(" ", "_") and kv.get("sources") == want:
            return float(kv["bytes_per_launch"])
    return None


def copy_calibration(args, torch, sync):
    """A plain device copy of known size: its HBM byte counters scale the
    dedispersion kernels' counters to bytes."""
    n = 1 << 28  # float32 elements: 1 GiB read and 1 GiB written per launch
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    ms, launch_ms, _ = time_steps(lambda: y.copy_(x), args.steps, args.warmup, sync)
    kms = float(np.mean(launch_ms))
    print(json.dumps({"metric": "device copy", "value": 2 * 4 * n / (kms / 1e3) / 1e9, "unit": "GB/s",
                      "bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n, "ms_per_step": ms,
                      "kernel_ms": kms, "steps": args.steps, "warmup": args.warmup}), flush=True)


WORKLOAD_TEXT = {
    "batched": "256 uneven beams in one persistent graph-captured launch (256/512/1024/1536 ch, "
               "1270-1570 MHz, 512-4096 DMs step 0.25, 8000-20000 samples, 50 us, FP32)",
    "apertif": "Apertif-like beam: 1024 ch 1270-1570 MHz, 2048 DMs step 0.25, 20000 samples, FP32",
    "lofar": "LOFAR-like beam: 32 ch 134.875-141.125 MHz, 2048 DMs step 0.01, 200000 samples, u8->i32",
    "diff": "32 Apertif-like beams, 1024 ch, 1024 DMs, 20000 samples: forward + adjoint + grad_w",
    "detect_apertif": "Apertif-like beam (as apertif) dedispersed and searched with boxcars of 1..32 "
                      "samples in one pass, series never stored",
    "detect_lofar": "LOFAR-like beam (as lofar) dedispersed and searched with boxcars of 1..32 "
                    "samples in one pass, series never stored",
}


def measure(wl, args, steps, warmup, plain_loop=True):
    """Prepare workload wl (inputs resident in HBM), tune or pin its kernels,
    time `steps` steps after `warmup` and return the JSON line as a dict."""
    import torch

    import paper_1601_01165_amd as dd
    import synth

    dev = torch.device("cuda:0")
    sync = torch.cuda.synchronize
    extra = {}
    if wl in ("batched", "apertif", "diff", "detect_apertif"):
        k = {"batched": 3, "apertif": 1, "diff": 4, "detect_apertif": 1}[wl]
    else:
        k = 2
    beams = synth.config(k)
    if args.beams:
        beams = beams[: args.beams]
    log(f"workload {wl}: {len(beams)} beam(s)")

    plans, xs, outs = [], [], []
    adds = 0
    algo_bytes = 0
    dm_samples = 0
    for i, b in enumerate(beams):
        p = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
        nin = b.nsamp + p.max_delay
        dtype = torch.uint8 if b.dtype == "u8" else torch.float32
        x = dd.empty_rows(1, b.nchan, nin, dtype, dev)
        if b.dtype == "u8":
            g = torch.Generator(device=dev)
            g.manual_seed(b.seed)
            v = torch.randn(x.shape, generator=g, device=dev)
            x.copy_(torch.clamp(torch.round(128.0 + 16.0 * v), 0, 255).to(torch.uint8))
            del v
        else:
            fill_noise(x, b.seed)
            delays = None
            for j, t0 in synth.pulses(b, p.max_delay):
                if delays is None:
                    delays = p.delays()
                inject_device(x[0], delays[j], t0, b.pulse_width, b.pulse_amp)
        out = dd.empty_rows(1, b.ndm, b.nsamp, torch.int32 if b.dtype == "u8" else torch.float32, dev)
        plans.append(p)
        xs.append(x)
        outs.append(out)
        adds += b.nchan * b.ndm * b.nsamp
        algo_bytes += b.nchan * nin * b.elem_bytes() + b.ndm * b.nsamp * 4 + 4 * b.nchan * b.ndm
        dm_samples += b.ndm * b.nsamp
        if i % 32 == 31:
            log(f"  prepared {i + 1} beams")
    sync()
    log(f"inputs resident: {sum(x.numel() * x.element_size() for x in xs) / 1e9:.2f} GB in, "
        f"{sum(o.numel() * 4 for o in outs) / 1e9:.2f} GB out")

    plain = None
    if wl == "batched":
        batch = dd.Batch(plans, xs, outs, tune=not args.no_tune and args.variant is None)
        if args.variant is not None:
            batch.set_variant(args.variant)
        if args.queues:
            batch.set_queues(args.queues)
        variant_name = dd.variant_names("f32")[batch.variant]
        extra["queues"] = batch.queues
        log(f"batch created: variant {batch.variant} {variant_name}, {batch.queues} work queue(s)")
        step = batch.execute
        if plain_loop and not args.no_plain:
            if not args.no_tune and args.variant is None:
                for i, (p, b) in enumerate(zip(plans, beams)):
                    p.autotune(1, b.nsamp, "f32")
                    if i % 64 == 63:
                        log(f"  tuned {i + 1} per-beam plans")
            ms_p, lp, _ = time_steps(batch.execute_per_beam, steps, warmup, sync)
            plain = {"value": dm_samples / (ms_p / 1e3), "ms_per_step": ms_p}
            log(f"plain per-beam loop: {ms_p:.3f} ms/step")
        kernel_name = "win_persistent"
    elif wl in ("apertif", "lofar"):
        p, b, x, o = plans[0], beams[0], xs[0], outs[0]
        wts = torch.ones(b.nchan, device=dev) if args.weights and b.dtype != "u8" else None
        if args.variant is not None:
            p.set_variant(args.variant, "u8" if b.dtype == "u8" else "f32")
            log(f"variant forced to {args.variant}")
        elif not args.no_tune:
            times = p.autotune(1, b.nsamp, "u8" if b.dtype == "u8" else "f32")
            extra["autotune_ms"] = {kk: round(v, 4) for kk, v in times.items()}
            log(f"autotuned: {times}")

        def step():
            dd.dedisperse(x, p, wts, nsamp=b.nsamp, out=o)
        dt = "u8" if b.dtype == "u8" else "f32"
        if wts is not None:
            extra["weights"] = "ones (fused multiply-add per term)"
        vi = p.variant(dt)
        variant_name = dd.variant_names(dt)[vi] if vi >= 0 else "direct"
        kernel_name = ("direct_u8_kernel" if dt == "u8" else "direct_f32_kernel") if vi < 0 else \
            ("u8s_kernel" if variant_name.startswith("u8s_") else "u8_kernel" if dt == "u8" else "win_kernel")
    elif wl in ("detect_apertif", "detect_lofar"):
        # single-pulse search fused into the dedispersion epilogue (boxcar
        # widths 1..32), the unfused path (store, then search) timed beside it
        p, b, x, o = plans[0], beams[0], xs[0], outs[0]
        dt = "u8" if b.dtype == "u8" else "f32"
        # room for the unfused path too (the dedispersed rows and their records)
        ws = torch.empty(b.ndm * (b.nsamp + 4) * 4 + (1 << 26), dtype=torch.uint8, device=dev)
        if args.variant is not None:
            p.set_variant(args.variant, dt)
            p.set_detect_variant(args.variant, dt)
        elif not args.no_tune:
            # the forward variant (used by the unfused path), then the search
            # path: every fused variant and the unfused one, the fastest kept
            p.autotune(1, b.nsamp, dt)
            fwd = p.variant(dt)
            extra["detect_tune_ms"] = {k: round(v, 4) for k, v in p.autotune_detect(1, b.nsamp, dt).items()}
            log(f"search paths: {extra['detect_tune_ms']}")
            chosen = p.detect_variant(dt)
            p.set_detect_variant(-1, dt)
            ms_u, _, _ = time_steps(lambda: dd.detect(x, p, nsamp=b.nsamp, workspace=ws), steps, warmup, sync)
            p.set_detect_variant(chosen, dt)
            extra["unfused_ms_per_step"] = ms_u
            extra["unfused_forward_variant"] = dd.variant_names(dt)[fwd] if fwd >= 0 else "direct"
            log(f"unfused (store, then search): {ms_u:.3f} ms/step")
        vi = p.detect_variant(dt)
        variant_name = dd.variant_names(dt)[vi] if vi >= 0 else "unfused"
        # algorithmic bytes: input once, delay table, the per-tile records and the results (no series)
        rec = dd.lib().dedisp_detect_workspace_bytes(p.handle, dd._dt(dt), 1, b.nsamp)
        algo_bytes = b.nchan * x.shape[2] * b.elem_bytes() + 4 * b.nchan * b.ndm + rec + 32 * b.ndm

        def step():
            dd.detect(x, p, nsamp=b.nsamp, workspace=ws)
        kernel_name = ("u8s_kernel" if dt == "u8" else "win_kernel") + " with the search epilogue + det_finish_kernel"
    else:  # diff: forward + adjoint with the weight gradient over all beams
        w = torch.ones(beams[0].nchan, device=dev)
        p0 = plans[0]
        xb = dd.empty_rows(len(beams), beams[0].nchan, xs[0].shape[2], torch.float32, dev)
        for i, x in enumerate(xs):
            xb[i].copy_(x[0])
        g = dd.empty_rows(len(beams), beams[0].ndm, beams[0].nsamp, torch.float32, dev)
        fill_noise(g, 5)
        ob = dd.empty_rows(len(beams), beams[0].ndm, beams[0].nsamp, torch.float32, dev)
        xs, outs = [xb], [ob]
        adds *= 2
        nin = xb.shape[2]
        if args.variant is not None:
            p0.set_variant(args.variant, "f32")
            p0.set_adjoint_variant(args.variant)
        elif not args.no_tune:
            p0.autotune(len(beams), beams[0].nsamp, "f32")
            times = p0.autotune_adjoint(len(beams), beams[0].nsamp)
            extra["adjoint_tune_ms"] = {k: round(v, 3) for k, v in times.items()}
            log(f"adjoint variants: {extra['adjoint_tune_ms']}")

        def step():
            dd.dedisperse(xb, p0, w, nsamp=beams[0].nsamp, out=ob)
            dd.adjoint(g, p0, nin, w, xb)
        kernel_name = "win_kernel (forward + adjoint)"
        fv, av = p0.variant("f32"), p0.adjoint_variant()
        variant_name = (f"{dd.variant_names('f32')[fv] if fv >= 0 else 'direct'} (forward), "
                        f"{dd.variant_names('f32')[av] if av >= 0 else 'direct'} (adjoint)")

    log("timing")
    ms, launch_ms, wall = time_steps(step, steps, warmup, sync)
    value = dm_samples / (ms / 1e3)
    kern_ms = float(np.mean(launch_ms))
    log(f"{ms:.3f} ms/step, {value:.4e} DM-trial*samples/s")
    cold = None
    if wl in ("apertif", "lofar", "detect_apertif", "detect_lofar") and not args.no_cold:
        # the inputs of these workloads fit the 256 MB MALL, so the warm steps
        # above may read them from it; these runs start from HBM
        cold_ms = float(np.median(time_cold(step, max(steps, 5), sync)))
        cold = {"runs": max(steps, 5), "ms_median": cold_ms, "value": dm_samples / (cold_ms / 1e3),
                "over_warm": cold_ms / ms,
                "note": "each run after a 512 MB scratch write (evicts the 256 MB MALL and the L2s), write not timed"}
        log(f"cold: {cold_ms:.3f} ms/step ({cold_ms / ms:.3f}x warm)")

    achieved = adds / (kern_ms / 1e3)
    roof = {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": ADD_PEAK / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / ADD_PEAK,
        "traffic": None,
        "kernel": kernel_name,
        "variant": variant_name,
        "kernel_ms": kern_ms,
        "note": "one FP32 add per (channel, DM trial, sample), the paper's flop count; peak = 157.3/2",
    }
    if wl == "lofar":
        roof.update({"bound": "hbm", "achieved": algo_bytes / (kern_ms / 1e3) / 1e9, "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": algo_bytes / (kern_ms / 1e3) / HBM_PEAK,
                     "note": "algorithmic bytes: input once + int32 output + delay table"})
        if cold:
            cold["roofline_frac"] = algo_bytes / (cold_ms / 1e3) / HBM_PEAK
    if wl.startswith("detect_"):
        roof["note"] = ("the paper's dedispersion adds only (one per channel, DM trial and sample); the search's "
                        "own integer/FP32 work is not counted; kernel_ms covers the tile kernel and the record merge")
        if "unfused_ms_per_step" in extra:
            extra["fused_over_unfused"] = extra["unfused_ms_per_step"] / ms
    roof["traffic"] = stored_traffic(wl, variant_name)
    roof["algorithmic_bytes"] = algo_bytes
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "DM-trial·samples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8" if wl in ("lofar", "detect_lofar") else "f32",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD_TEXT[wl],
            "beams": len(beams),
            "dm_trial_samples_per_step": dm_samples,
            "adds_per_step": adds,
        },
        "gbps": algo_bytes / (ms / 1e3) / 1e9,
        "hbm_frac": algo_bytes / (ms / 1e3) / HBM_PEAK,
        "valu_frac": adds / (ms / 1e3) / ADD_PEAK,
        "gflops_paper_convention": adds / (ms / 1e3) / 1e9,
        # seconds of observed data (summed over beams) dedispersed per second
        # of compute; the paper's real-time criterion is >= 1 per beam
        "realtime_factor": sum(b.nsamp * b.tsamp_s for b in beams) / (ms / 1e3),
        "roofline": roof,
    }
    if cold:
        line["cold"] = cold
    if plain:
        line["plain_value"] = plain["value"]
        line["plain_ms_per_step"] = plain["ms_per_step"]
        line["batched_over_plain"] = value / plain["value"]
    line.update(extra)
    return line, beams


def secondary(wl, args):
    """The LOFAR-like (uint8, HBM-bound) and differentiable workloads timed
    after the headline one, in the same process: their own roofline, variant
    and kernel time, in a compact object."""
    import torch

    steps, warmup = {"lofar": (200, 10), "diff": (5, 2)}[wl]
    line, _ = measure(wl, args, steps, warmup, plain_loop=False)
    keep = ("value", "unit", "ms_per_step", "steps", "warmup", "dtype", "config", "gbps", "hbm_frac", "valu_frac",
            "roofline", "cold", "autotune_ms", "adjoint_tune_ms")
    out = {k: line[k] for k in keep if k in line}
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build runs on one GPU only: beams are independent and shard by beam "
                                   "with no exchange; run one process per GPU with a share of the beams"}))
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(torch.device("cuda:0"))
    wl = args.workload
    if wl == "copy":
        copy_calibration(args, torch, torch.cuda.synchronize)
        return
    line, beams = measure(wl, args, args.steps, args.warmup)
    line["paper_context"] = {
        "hd7970_apertif_2000dm": "0.08 s per 1 s of data = 5.0e8 DM-trial*samples/s (AMD HD7970, OpenCL, FP32)"}
    if wl == "batched" and not args.no_secondary and not args.beams:
        # the headline's inputs and outputs (56 GB) are released first
        import gc

        gc.collect()
        torch.cuda.empty_cache()
        line["secondary"] = {w: secondary(w, args) for w in ("lofar", "diff")}
    if not args.no_cpu:
        log("CPU oracle baseline")
        if wl == "batched" and not args.beams:
            line["cpu_baseline"] = cpu_baseline_subset(beams, args.cpu_seconds)
        else:
            line["cpu_baseline"] = cpu_baseline(beams[0], args.cpu_seconds, search=wl.startswith("detect_"))
        log(f"cpu baseline {line['cpu_baseline']['value']:.3e}")
    if not args.no_cpu_tuned and not wl.startswith("detect_"):
        log("tuned CPU comparator")
        line["cpu_tuned"] = cpu_tuned(beams[0], args.cpu_tuned_seconds)
        line["gpu_over_cpu_tuned"] = line["value"] / line["cpu_tuned"]["value"]
        log(f"tuned cpu {line['cpu_tuned']['value']:.3e}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
