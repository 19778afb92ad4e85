"""Pins of the oracle's single-pulse search (boxcar S/N over dedispersed
series, the detection step that follows dedispersion in the real-time
pipeline of Section 1).

The oracle sums each window directly with NumPy; the pins are closed forms of
a rectangular pulse on a flat background, a brute force in plain Python
loops, the width-1 case against the separately pinned max-minus-mean S/N, the
invariance of S/N and of the chosen window under positive affine maps, the
degenerate constant row, and recovery of an injected pulse through the whole
dedispersion chain.
"""
import math

import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("W,A,n,t0", [(1, 3.0, 50, 7), (2, 1.5, 64, 0), (4, 5.0, 100, 60), (8, 5.0, 100, 40),
                                      (16, 2.0, 300, 284), (32, 0.5, 1000, 123)])
def test_rectangular_pulse_closed_form(W, A, n, t0):
    # A pulse of width W and height A on zeros: mean = W A / n,
    # var = W A^2 / n - mean^2.  A window of width w <= W reaches w A first at
    # t0, so S/N_w = sqrt(w) (A - mean) / std grows with w up to W; a wider
    # window holds at most W A, S/N_w = (W A - w mean) / (std sqrt(w)), which
    # falls again.  So the search returns width W at t0.
    y = np.zeros(n)
    y[t0:t0 + W] = A
    mean = W * A / n
    std = math.sqrt(W * A * A / n - mean * mean)
    for kmax in range(7):
        wmax = 1 << kmax
        snr, width, start, m, s = oracle.detect_row(y, kmax + 1)
        wexp = min(W, wmax)
        assert width == wexp and start == t0
        assert snr == pytest.approx(math.sqrt(wexp) * (A - mean) / std, rel=1e-12)
        assert m == pytest.approx(mean, rel=1e-14) and s == pytest.approx(std, rel=1e-12)
    # wider windows: first start that still covers the whole pulse
    for w in (2 * W, 4 * W):
        if w <= n:
            b = oracle.boxcar_sums(y, w)
            assert b.max() == pytest.approx(W * A) and int(np.argmax(b)) == max(0, t0 + W - w)


def _brute(y, nwidth):
    y = [float(v) for v in y]
    n = len(y)
    mean = sum(y) / n
    std = math.sqrt(sum((v - mean) ** 2 for v in y) / n)
    best = None
    w = 1
    for _ in range(nwidth):
        if w > n:
            break
        top, at = None, None
        for t in range(n - w + 1):
            s = 0.0
            for i in range(w):
                s += y[t + i]
            if top is None or s > top:
                top, at = s, t
        snr = (top - w * mean) / (std * math.sqrt(w)) if std > 0 else 0.0
        if best is None or snr > best[0]:
            best = (snr, w, at)
        w *= 2
    return best + (mean, std)


@pytest.mark.parametrize("n", [1, 2, 5, 33, 64, 97])
@pytest.mark.parametrize("nwidth", [1, 3, 6])
def test_bruteforce_tiny(n, nwidth):
    rng = np.random.default_rng(n * 7 + nwidth)
    for kind in ("normal", "ints"):
        y = rng.standard_normal(n) if kind == "normal" else rng.integers(0, 9, n).astype(float)
        got = oracle.detect_row(y, nwidth)
        ref = _brute(y, nwidth)
        assert got[1:3] == ref[1:3], (kind, got, ref)
        for a, b in zip((got[0],) + got[3:], (ref[0],) + ref[3:]):
            assert a == pytest.approx(b, rel=1e-9, abs=1e-12)


def test_width1_is_max_minus_mean_snr():
    rng = np.random.default_rng(5)
    for n in (10, 1000, 4097):
        y = rng.standard_normal(n)
        snr, width, start, _, _ = oracle.detect_row(y, 1)
        assert width == 1 and start == int(np.argmax(y))
        assert snr == pytest.approx(oracle.snr(y), rel=1e-12)


def test_affine_invariance():
    rng = np.random.default_rng(11)
    y = rng.standard_normal(2000)
    y[700:704] += 3.0
    r0 = oracle.detect_row(y, 6)
    for a, b in ((2.0, 0.0), (0.25, -7.0), (13.0, 1e3)):
        r1 = oracle.detect_row(a * y + b, 6)
        assert r1[1:3] == r0[1:3]
        assert r1[0] == pytest.approx(r0[0], rel=1e-9)
        assert r1[3] == pytest.approx(a * r0[3] + b, rel=1e-12)
        assert r1[4] == pytest.approx(a * r0[4], rel=1e-12)


def test_constant_row_is_degenerate():
    for n in (1, 3, 100):
        assert oracle.detect_row(np.full(n, 4.0), 6) == (0.0, 1, 0, 4.0, 0.0)


def test_pulse_recovered_through_dedispersion():
    # Noise-free config-0 geometry: the injected DM row holds the pulse whole
    # (width 4 at t0 = 2048) and has the largest S/N of all rows.
    b = synth.config(0)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    x = np.zeros((b.nchan, nin), np.float32)
    (j0, t0), = synth.pulses(b, int(delta.max()))
    synth.inject(x, delta, j0, t0, b.pulse_width, b.pulse_amp)
    r = oracle.detect(oracle.forward_f32(x, delta, b.nsamp), 6)
    assert int(np.argmax(r["snr"][0])) == j0
    assert r["width"][0, j0] == b.pulse_width and r["start"][0, j0] == t0
    # noisy: still the top row, at the injected width and start
    x = synth.noise(b, nin)
    synth.inject(x, delta, j0, t0, b.pulse_width, b.pulse_amp)
    r = oracle.detect(oracle.forward_f32(x, delta, b.nsamp), 6)
    assert int(np.argmax(r["snr"][0])) == j0
    assert r["width"][0, j0] == b.pulse_width and r["start"][0, j0] == t0
