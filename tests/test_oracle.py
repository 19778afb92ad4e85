"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks it against a
hand-worked value of Equation 1, a number the paper prints, a closed form, an
invariant, a special case that reduces to a library routine (NumPy sums and
dense matrix products), or the transpose identity.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth


# ---------------------------------------------------------------------------
# Delay law (Section 2, Equation 1)
# ---------------------------------------------------------------------------

def _read_eq1(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "eq1_hand_values.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            case, flo, fhi, ts, dm, x, d = line.split()
            rows.append((case, float(flo), float(fhi), float(ts), float(dm), float(x), int(d)))
    return rows


def test_delay_hand_worked_values(golden_dir):
    rows = _read_eq1(golden_dir)
    assert len(rows) >= 10
    for case, flo, fhi, ts, dm, x_exact, d_exact in rows:
        x = oracle.delay_samples([flo, fhi], ts, [dm])
        d = oracle.delay_table([flo, fhi], ts, [dm])
        assert x[0, 0] == pytest.approx(x_exact, rel=1e-12, abs=1e-12), (case, dm)
        assert d[0, 0] == d_exact, (case, dm)
        assert d[0, 1] == 0  # top of the band
        # channel order does not matter: the band top is the maximum frequency
        d2 = oracle.delay_table([fhi, flo], ts, [dm])
        assert d2[0, 0] == 0 and d2[0, 1] == d_exact


@pytest.mark.parametrize("k", [0, 1, 2])
def test_delay_invariants(k):
    b = synth.config(k)[0]
    f = b.freqs()
    d = oracle.delay_table(f, b.tsamp_s, b.dms())
    assert d.dtype == np.int32 and d.shape == (b.ndm, b.nchan)
    assert (d[0] == 0).all()  # DM 0
    assert (d[:, np.argmax(f)] == 0).all()  # top channel
    assert (d >= 0).all()
    assert (np.diff(d, axis=0) >= 0).all()  # non-decreasing in DM (DMs ascending)
    assert (np.diff(d, axis=1) <= 0).all()  # non-increasing in frequency (ascending channels)
    # Eq. 1 is linear in DM: doubling DM doubles the unrounded delay, so the
    # rounded delays differ by at most one sample.
    half = np.arange(0, b.ndm // 2)
    assert (np.abs(d[2 * half] - 2 * d[half]) <= 1).all()


def test_delay_config0_worked_values():
    # Config 0 geometry, lowest channel centre 1400.78125 MHz, top 1499.21875 MHz.
    b = synth.config(0)[0]
    x = oracle.delay_samples(b.freqs(), b.tsamp_s, b.dms())
    d = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    assert abs(x[17, 0] - 91.330311) < 1e-6 and d[17, 0] == 91
    assert abs(x[31, 0] - 166.543509) < 1e-6 and d[31, 0] == 167
    assert int(d[17].sum()) == 2824
    assert [int(d[j].sum()) for j in range(5)] == [0, 166, 334, 501, 663]


@pytest.mark.parametrize("k", [0, 1, 2])
def test_delay_rounding_margin(k):
    # No unrounded delay lies within 1e-9 samples of a rounding boundary, so
    # any correct FP64 evaluation gives the same integer table.
    b = synth.config(k)[0]
    x = oracle.delay_samples(b.freqs(), b.tsamp_s, b.dms())
    frac = x - np.floor(x)
    nz = x[x > 0]
    fr = nz - np.floor(nz)
    assert np.min(np.abs(fr - 0.5)) > 1e-9
    assert frac.min() >= 0


def test_delay_invalid_arguments():
    with pytest.raises(ValueError):
        oracle.delay_table([1400.0], 0.0, [1.0])
    with pytest.raises(ValueError):
        oracle.delay_table([1400.0, -5.0], 1e-3, [1.0])
    with pytest.raises(ValueError):
        oracle.delay_table([1400.0], 1e-3, [-1.0])
    with pytest.raises(ValueError):
        oracle.delay_table([1400.0, float("nan")], 1e-3, [1.0])
    with pytest.raises(ValueError):
        oracle.delay_table([1.0, 1e9], 1e-9, [1e6])  # delay overflows int32


def test_paper_printed_work_and_rates(golden_dir):
    vals = {}
    with open(os.path.join(golden_dir, "paper_numbers.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, *v = line.split()
                vals[k] = [float(t) for t in v]
    # Work per DM: one add per (channel, output sample); the paper rounds to MFLOP.
    for key, (k_sel) in (("work_per_dm_apertif", 1), ("work_per_dm_lofar", 2)):
        c, s, mflop = vals[key]
        b = synth.config(k_sel)[0]
        assert (b.nchan, b.nsamp) == (c, s)
        assert round(c * s / 1e6) == mflop
        # the oracle performs exactly c adds per output element: check on a
        # DM row of all-ones input, whose every output equals c
        x = np.ones((int(c), 64 + 8), np.float32)
        out = oracle.forward_f32(x, np.zeros((1, int(c)), np.int32), 64)
        assert (out == c).all()
    n, d, s, c, tf = vals["tflops_apertif_450"]
    assert abs(n * d * s * c / 1e12 - tf) < 0.1  # 18.43 against the printed 18.5
    n, c, s, e, g = vals["rate_in_gbs"]
    assert round(n * c * s * e / 1e9) in (g, g + 1)
    n, d, s, e, g = vals["rate_out_gbs"]
    assert round(n * d * s * e / 1e9) == g


# ---------------------------------------------------------------------------
# Forward dedispersion (Section 2.1, Algorithm 1)
# ---------------------------------------------------------------------------

def _dense(delta, nsamp, nin, w=None):
    """Dense matrix of the forward map: out[j*S+s] = sum M[j*S+s, c*nin+t] x[c, t]."""
    nd, nc = delta.shape
    M = np.zeros((nd * nsamp, nc * nin))
    for j in range(nd):
        for s in range(nsamp):
            for c in range(nc):
                M[j * nsamp + s, c * nin + s + delta[j, c]] += 1.0 if w is None else w[c]
    return M


def _rand_case(rng, nc, nd, ns, maxd):
    delta = rng.integers(0, maxd + 1, size=(nd, nc)).astype(np.int32)
    nin = ns + int(delta.max()) + int(rng.integers(0, 3))
    return delta, nin


@pytest.mark.parametrize("seed", range(6))
def test_forward_dense_bruteforce(seed):
    rng = np.random.default_rng(seed)
    nc, nd, ns = int(rng.integers(1, 9)), int(rng.integers(1, 7)), int(rng.integers(1, 33))
    delta, nin = _rand_case(rng, nc, nd, ns, 12)
    nb = int(rng.integers(1, 3))
    x = synth.small_ints(rng, (nb, nc, nin))
    w = synth.small_ints(rng, nc, -3, 3)
    for wv in (None, w):
        M = _dense(delta, ns, nin, wv)
        ref = np.stack([(M @ x[b].reshape(-1).astype(np.float64)).reshape(nd, ns) for b in range(nb)])
        out = oracle.forward_f32(x, delta, ns, wv)
        assert np.array_equal(out.astype(np.float64), ref)  # small integers: exact in FP32
        out64 = oracle.forward_f64(x, delta, ns, wv)
        assert np.array_equal(out64, ref)
    # real-valued data in FP64 against the dense product
    xr = rng.standard_normal((nb, nc, nin))
    M = _dense(delta, ns, nin, w)
    ref = np.stack([(M @ xr[b].reshape(-1)).reshape(nd, ns) for b in range(nb)])
    np.testing.assert_allclose(oracle.forward_f64(xr, delta, ns, w), ref, rtol=1e-12, atol=1e-12)


def test_forward_fp32_within_summation_bound():
    rng = np.random.default_rng(3)
    nc, nd, ns = 300, 5, 200
    delta, nin = _rand_case(rng, nc, nd, ns, 40)
    x = rng.standard_normal((1, nc, nin)).astype(np.float32)
    w = (1.0 + 0.1 * rng.standard_normal(nc)).astype(np.float32)
    o32 = oracle.forward_f32(x, delta, ns, w).astype(np.float64)
    o64, scale = oracle.forward_f64(x.astype(np.float64), delta, ns, w.astype(np.float64), with_scale=True)
    # sequential FP32 sum of rounded products: |err| <= (nc + 1) * u * sum |w x| (u = 2^-24)
    assert (np.abs(o32 - o64) <= (nc + 1) * 2.0 ** -24 * scale).all()
    assert np.abs(o32 - o64).max() > 0  # FP32 really is FP32


@pytest.mark.parametrize("weighted", [False, True])
def test_forward_fp32_order_per_output_bruteforce(weighted):
    """Each output is the sequential FP32 sum of its terms in ascending channel
    order (Section 2.1, single precision): a pure-Python loop over one output
    at a time, on real-valued data where the order changes the rounding.  A
    weighted term is the FP32 product w * x, rounded, then added (the weight
    is a gain on the data); with real-valued weights a fused multiply-add
    rounds differently somewhere, which the loop would catch."""
    rng = np.random.default_rng(21)
    nc, nd, ns, nb = 9, 5, 23, 2
    delta, nin = _rand_case(rng, nc, nd, ns, 10)
    x = (rng.standard_normal((nb, nc, nin)) * 10.0 ** rng.integers(-3, 4, (nb, nc, nin))).astype(np.float32)
    w = rng.uniform(0.3, 3.0, nc).astype(np.float32) if weighted else None
    out = oracle.forward_f32(x, delta, ns, w)
    fused_differs = False
    for b in range(nb):
        for j in range(nd):
            for t in range(ns):
                acc = np.float32(0.0)
                facc = 0.0
                for c in range(nc):
                    term = x[b, c, t + delta[j, c]]
                    if w is not None:
                        # the fused form: w * x + acc exactly, then one rounding
                        facc = float(np.float32(float(w[c]) * float(term) + float(facc)))
                        term = np.float32(w[c] * term)
                    acc = np.float32(acc + term)
                assert out[b, j, t] == acc, (b, j, t)
                fused_differs |= w is not None and np.float32(facc) != acc
    if weighted:
        assert fused_differs  # the data tells the two roundings apart
    # a different channel order rounds differently somewhere (the pin can fail)
    rev = oracle.forward_f32(x[:, ::-1].copy(), delta[:, ::-1].copy(), ns, None if w is None else w[::-1].copy())
    assert not np.array_equal(rev, out)


def test_forward_weights_are_a_gain_on_the_input():
    """Weighted dedispersion equals unweighted dedispersion of the input with
    every channel row scaled by its weight in FP32 (the weight is a per-channel
    gain), bit for bit, at the config-0 geometry with real-valued weights."""
    rng = np.random.default_rng(22)
    b = synth.config(0)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    x = rng.standard_normal((2, b.nchan, nin)).astype(np.float32)
    w = rng.uniform(0.25, 2.0, b.nchan).astype(np.float32)
    scaled = (w[None, :, None] * x).astype(np.float32)
    assert np.array_equal(oracle.forward_f32(x, delta, b.nsamp, w), oracle.forward_f32(scaled, delta, b.nsamp))
    pb = rng.integers(0, 2, 300).astype(np.int32)
    pd = rng.integers(0, b.ndm, 300).astype(np.int32)
    ps = rng.integers(0, b.nsamp, 300).astype(np.int32)
    got, _ = oracle.forward_points(x, delta, pb, pd, ps, w)
    ref, _ = oracle.forward_points(scaled, delta, pb, pd, ps)
    assert np.array_equal(got, ref)


def test_forward_dm0_is_channel_sum():
    rng = np.random.default_rng(1)
    b = synth.config(0)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    x = synth.small_ints(rng, (b.nchan, nin))
    out = oracle.forward_f32(x, delta, b.nsamp)
    assert np.array_equal(out[0, 0], x[:, :b.nsamp].sum(axis=0))


def test_forward_all_zero_dms_rows_identical():
    # Section 4.3: with every DM trial 0 all trials read the same data.
    b = synth.config(1)[0]
    f = b.freqs()[::16]
    delta = oracle.delay_table(f, b.tsamp_s, np.zeros(7))
    assert (delta == 0).all()
    rng = np.random.default_rng(2)
    x = rng.standard_normal((f.size, 300)).astype(np.float32)
    out = oracle.forward_f32(x, delta, 300)
    for j in range(1, 7):
        assert np.array_equal(out[0, j], out[0, 0])


def test_forward_single_channel_is_copy():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((1, 1, 500)).astype(np.float32)
    delta = np.array([[0], [7], [100]], np.int32)
    out = oracle.forward_f32(x, delta, 400)
    for j, d in enumerate((0, 7, 100)):
        assert np.array_equal(out[0, j], x[0, 0, d:d + 400])


def test_forward_constant_and_ramp_and_onehot():
    b = synth.config(0)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    C = b.nchan
    # constant input: every output is the sum of the weights
    w = np.arange(1, C + 1, dtype=np.float32) / 8
    out = oracle.forward_f32(np.full((C, nin), 2.0, np.float32), delta, b.nsamp, w)
    assert (out == np.float32(2.0 * w.astype(np.float64).sum())).all()
    # ramp in[c][t] = t: out[j][t] = C*t + sum_c delta[j][c]  (config 0, DM 17: 64 t + 2824)
    ramp = np.tile(np.arange(nin, dtype=np.float32), (C, 1))
    out = oracle.forward_f32(ramp, delta, b.nsamp)
    t = np.arange(b.nsamp)
    for j in range(b.ndm):
        assert np.array_equal(out[0, j], (C * t + int(delta[j].sum())).astype(np.float32))
    assert np.array_equal(out[0, 17], (64 * t + 2824).astype(np.float32))
    # one-hot channel k: out[j][t] = in[k][t + delta[j][k]]
    rng = np.random.default_rng(5)
    k = 9
    x = np.zeros((C, nin), np.float32)
    x[k] = rng.standard_normal(nin).astype(np.float32)
    out = oracle.forward_f32(x, delta, b.nsamp)
    for j in range(b.ndm):
        assert np.array_equal(out[0, j], x[k, delta[j, k]:delta[j, k] + b.nsamp])


def test_forward_linearity():
    rng = np.random.default_rng(6)
    nc, nd, ns = 17, 9, 123
    delta, nin = _rand_case(rng, nc, nd, ns, 30)
    x = synth.small_ints(rng, (nc, nin))
    y = synth.small_ints(rng, (nc, nin))
    a, bb = 3.0, -2.0
    lhs = oracle.forward_f32((a * x + bb * y).astype(np.float32), delta, ns)
    rhs = a * oracle.forward_f32(x, delta, ns) + bb * oracle.forward_f32(y, delta, ns)
    assert np.array_equal(lhs, rhs.astype(np.float32))


def test_forward_pulse_recovery_noise_free():
    b = synth.config(0)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    x = np.zeros((b.nchan, nin), np.float32)
    (j0, t0), = synth.pulses(b, int(delta.max()))
    synth.inject(x, delta, j0, t0, b.pulse_width, b.pulse_amp)
    out = oracle.forward_f32(x, delta, b.nsamp)[0]
    assert j0 == 17 and t0 == 2048
    assert (out[17, 2048:2052] == 320.0).all()
    peak = out.max(axis=1)
    assert peak[17] == 320.0 and (np.delete(peak, 17) < 320.0).all()


def test_forward_pulse_recovery_noisy():
    b = synth.config(0)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    x = synth.noise(b, nin)
    for j0, t0 in synth.pulses(b, int(delta.max())):
        synth.inject(x, delta, j0, t0, b.pulse_width, b.pulse_amp)
    out = oracle.forward_f32(x, delta, b.nsamp)[0]
    s = [oracle.snr(out[j]) for j in range(b.ndm)]
    assert int(np.argmax(s)) == 17
    assert int(np.argmax(out[17])) in range(2048, 2052)


def test_forward_pulse_recovery_config1_geometry():
    # Apertif-like band, a subset of channels; each pulse peaks at its own DM.
    b = synth.config(1)[0]
    f = b.freqs()[::8]
    dms = b.dms()[:256]
    delta = oracle.delay_table(f, b.tsamp_s, dms)
    ns = 2000
    nin = ns + int(delta.max())
    rng = np.random.default_rng(8)
    x = (0.3 * rng.standard_normal((f.size, nin))).astype(np.float32)
    picks = [(40, 300), (120, 900), (250, 1500)]
    for j0, t0 in picks:
        synth.inject(x, delta, j0, t0, 4, 1.0)
    out = oracle.forward_f32(x, delta, ns)[0]
    for j0, t0 in picks:
        seg = out[:, t0:t0 + 4].sum(axis=1)
        assert abs(int(np.argmax(seg)) - j0) <= 1
        assert out[j0, t0:t0 + 4].min() > 0.8 * f.size


def test_forward_u8_matches_integer_f32():
    rng = np.random.default_rng(9)
    nc, nd, ns = 32, 12, 300
    delta, nin = _rand_case(rng, nc, nd, ns, 60)
    x = rng.integers(0, 256, size=(2, nc, nin)).astype(np.uint8)
    o8 = oracle.forward_u8(x, delta, ns)
    M = _dense(delta, ns, nin)
    for b in range(2):
        ref = (M @ x[b].reshape(-1).astype(np.float64)).reshape(nd, ns)
        assert np.array_equal(o8[b].astype(np.float64), ref)
    assert o8.dtype == np.int32


def test_forward_points_match_full():
    rng = np.random.default_rng(10)
    nc, nd, ns = 40, 9, 257
    delta, nin = _rand_case(rng, nc, nd, ns, 50)
    x = rng.standard_normal((3, nc, nin)).astype(np.float32)
    w = rng.uniform(0.5, 1.5, nc).astype(np.float32)
    full = oracle.forward_f32(x, delta, ns, w)
    pb = rng.integers(0, 3, 500)
    pd = rng.integers(0, nd, 500)
    ps = rng.integers(0, ns, 500)
    v, sc = oracle.forward_points(x, delta, pb, pd, ps, w)
    assert np.array_equal(v, full[pb, pd, ps])
    _, scale = oracle.forward_f64(x.astype(np.float64), delta, ns, w.astype(np.float64), with_scale=True)
    np.testing.assert_allclose(sc, scale[pb, pd, ps], rtol=1e-12)
    xu = rng.integers(0, 256, size=(3, nc, nin)).astype(np.uint8)
    fu = oracle.forward_u8(xu, delta, ns)
    vu, _ = oracle.forward_points(xu, delta, pb, pd, ps)
    assert np.array_equal(vu, fu[pb, pd, ps])


# ---------------------------------------------------------------------------
# Adjoint and weight gradient (transpose of the Algorithm 1 map)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_adjoint_dense_transpose_and_dot_identity(seed):
    rng = np.random.default_rng(100 + seed)
    nc, nd, ns = int(rng.integers(1, 8)), int(rng.integers(1, 6)), int(rng.integers(1, 30))
    delta, nin = _rand_case(rng, nc, nd, ns, 10)
    w = synth.small_ints(rng, nc, -3, 3)
    g = synth.small_ints(rng, (1, nd, ns))
    M = _dense(delta, ns, nin, w)
    ref = (M.T @ g[0].reshape(-1).astype(np.float64)).reshape(nc, nin)
    got = oracle.adjoint_gather_f32(g, delta, nin, w)[0]
    assert np.array_equal(got.astype(np.float64), ref)
    # <A x, y> == <x, A^T y>, exact on integer data
    x = synth.small_ints(rng, (1, nc, nin))
    lhs = float((oracle.forward_f32(x, delta, ns, w).astype(np.float64) * g.astype(np.float64)).sum())
    rhs = float((x.astype(np.float64) * got.astype(np.float64)).sum())
    assert lhs == rhs


def test_adjoint_gather_equals_scatter_bitwise():
    rng = np.random.default_rng(7)
    b = synth.config(0)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    g = rng.standard_normal((2, b.ndm, b.nsamp)).astype(np.float32)
    w = rng.uniform(0.5, 2.0, b.nchan).astype(np.float32)
    ga = oracle.adjoint_gather_f32(g, delta, nin, w)
    sc = oracle.adjoint_scatter_f32(g, delta, nin, w)
    assert np.array_equal(ga, sc)
    G64, A = oracle.adjoint_gather_f64(g, delta, nin)
    assert (np.abs(ga / w[None, :, None] - G64) <= b.ndm * 2.0 ** -24 * A + 1e-30).all()
    # out-of-range terms contribute nothing: inputs past nsamp + max delay of a
    # channel get no gradient; the last input sample of the top channel gets none
    assert (ga[:, np.argmax(b.freqs()), b.nsamp:] == 0).all()


def test_grad_w_finite_differences():
    rng = np.random.default_rng(12)
    nc, nd, ns = 11, 7, 90
    delta, nin = _rand_case(rng, nc, nd, ns, 25)
    x = rng.standard_normal((2, nc, nin)).astype(np.float32)
    g = rng.standard_normal((2, nd, ns)).astype(np.float32)
    w = rng.uniform(0.5, 1.5, nc)
    gw, scale = oracle.grad_w(x, g, delta)

    def L(wv):
        return float((oracle.forward_f64(x.astype(np.float64), delta, ns, wv) * g.astype(np.float64)).sum())

    eps = 1e-3
    for c in range(nc):
        e = np.zeros(nc)
        e[c] = eps
        fd = (L(w + e) - L(w - e)) / (2 * eps)
        assert abs(fd - gw[c]) <= 1e-9 * scale[c] + 1e-9
    # and against the adjoint: grad_w[c] = sum_b,t x[b][c][t] * G[b][c][t]
    G = oracle.adjoint_gather_f64(g, delta, nin)[0]
    np.testing.assert_allclose(gw, (x.astype(np.float64) * G).sum(axis=(0, 2)), rtol=1e-10, atol=1e-10)


# ---------------------------------------------------------------------------
# S/N and the loss of the differentiable workload
# ---------------------------------------------------------------------------

def test_snr_hand_value_and_gradient():
    assert oracle.snr([0.0, 0.0, 0.0, 4.0]) == pytest.approx(math.sqrt(3.0), rel=1e-15)
    rng = np.random.default_rng(13)
    y = rng.standard_normal(50)
    y[17] += 6.0
    g = oracle.snr_grad(y)
    eps = 1e-6
    for i in (0, 17, 33):
        e = np.zeros_like(y)
        e[i] = eps
        fd = (oracle.snr(y + e) - oracle.snr(y - e)) / (2 * eps)
        assert abs(fd - g[i]) < 1e-6


def test_loss_gradient_chain_finite_differences():
    # d loss / d w and d loss / d x through the forward map, the S/N gradient and
    # the adjoint, against central differences of the FP64 loss (config 0 geometry).
    b = synth.config(0)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    ns = 512
    nin = ns + int(delta.max())
    rng = np.random.default_rng(14)
    x = rng.standard_normal((1, b.nchan, nin))
    synth.inject(x[0], delta, 17, 200, 4, 5.0)
    w = rng.uniform(0.8, 1.2, b.nchan)
    picks = [(0, 17), (0, 5)]

    def loss(xv, wv):
        return oracle.snr_loss(oracle.forward_f64(xv, delta, ns, wv), picks)

    out = oracle.forward_f64(x, delta, ns, w)
    g = np.zeros_like(out)
    for bb, j in picks:
        g[bb, j] -= oracle.snr_grad(out[bb, j]) / len(picks)
    G = oracle.adjoint_gather_f64(g, delta, nin)[0]
    gw = (x * G).sum(axis=(0, 2))
    gx = w[None, :, None] * G
    eps = 1e-3
    for c in range(0, b.nchan, 7):
        e = np.zeros_like(w)
        e[c] = eps
        fd = (loss(x, w + e) - loss(x, w - e)) / (2 * eps)
        assert abs(fd - gw[c]) < 1e-5 * max(1.0, abs(gw[c]))
    for (c, t) in [(0, 200 + int(delta[17, 0])), (63, 201), (30, 10), (5, 400)]:
        e = np.zeros_like(x)
        e[0, c, t] = eps
        fd = (loss(x + e, w) - loss(x - e, w)) / (2 * eps)
        assert abs(fd - gx[0, c, t]) < 1e-6 * max(1.0, abs(gx[0, c, t])) + 1e-8
