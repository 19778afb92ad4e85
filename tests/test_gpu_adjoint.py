"""GPU parity of the adjoint, the weight gradient and autograd.

The adjoint sums DM trials in ascending order with FP32 adds and scales by
w[c] once, as the oracle's gather form does, so grad_in is expected
bit-identical; grad_w is checked against the oracle's FP64 definition within
1e-5 of sum |g * x|.  Autograd gradients of the S/N loss are checked against
the oracle's FP64 chain and against central finite differences.
"""
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


def _rows(x, dtype=torch.float32):
    dd = _dd()
    t = dd.empty_rows(x.shape[0], x.shape[1], x.shape[2], dtype, "cuda", zero=True)
    t.copy_(torch.from_numpy(np.ascontiguousarray(x)))
    return t


def _adj_variants(plan):
    dd = _dd()
    out = [-1]
    for i in range(len(dd.variant_names("f32"))):
        try:
            plan.set_adjoint_variant(i)
            out.append(i)
        except dd.DedispError:
            pass
    return out


@pytest.mark.parametrize("weighted", [False, True])
def test_adjoint_config0(weighted):
    dd = _dd()
    b = synth.config(0)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    rng = np.random.default_rng(21)
    nb = 2
    g = rng.standard_normal((nb, b.ndm, b.nsamp)).astype(np.float32)
    x = rng.standard_normal((nb, b.nchan, nin)).astype(np.float32)
    w = rng.uniform(0.5, 1.5, b.nchan).astype(np.float32) if weighted else None
    ref_gi = oracle.adjoint_gather_f32(g, delta, nin, w)
    ref_gw, scale = oracle.grad_w(x, g, delta)
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    gg, xg = _rows(g), _rows(x)
    wg = torch.from_numpy(w).cuda() if weighted else None
    vs = _adj_variants(plan)
    assert len(vs) >= 2
    for v in vs:
        _note(f"adjoint config0 weighted={weighted} variant {v}")
        plan.set_adjoint_variant(v)
        gi, gw = dd.adjoint(gg, plan, nin, wg, xg)
        torch.cuda.synchronize()
        gi = gi.cpu().numpy()
        assert np.array_equal(gi, ref_gi), f"grad_in differs (variant {v}), max {np.abs(gi - ref_gi).max()}"
        gw = gw.cpu().numpy().astype(np.float64)
        assert (np.abs(gw - ref_gw) <= 1e-5 * scale + 1e-6 * np.abs(ref_gw)).all(), f"grad_w variant {v}"


def test_adjoint_scatter_agrees_and_ragged():
    dd = _dd()
    rng = np.random.default_rng(22)
    for nc, nd, ns, order in [(1, 1, 1, "asc"), (7, 3, 130, "desc"), (64, 37, 1029, "shuffled"), (130, 70, 700, "asc")]:
        f = 1270 + (np.arange(nc) + 0.5) * 300 / nc
        dms = np.arange(nd) * 0.25
        if order == "desc":
            f = f[::-1].copy()
        elif order == "shuffled":
            dms = rng.permutation(dms)
        delta = oracle.delay_table(f, 5e-5, dms)
        nin = ns + int(delta.max()) + 2
        g = rng.standard_normal((1, nd, ns)).astype(np.float32)
        x = rng.standard_normal((1, nc, nin)).astype(np.float32)
        ref = oracle.adjoint_scatter_f32(g, delta, nin)
        ref_gw, scale = oracle.grad_w(x, g, delta)
        plan = dd.Plan(f, 5e-5, dms)
        for v in _adj_variants(plan):
            _note(f"adjoint ragged {(nc, nd, ns, order)} variant {v}")
            plan.set_adjoint_variant(v)
            gi, gw = dd.adjoint(_rows(g), plan, nin, None, _rows(x))
            torch.cuda.synchronize()
            assert np.array_equal(gi.cpu().numpy(), ref), (nc, nd, ns, v)
            assert (np.abs(gw.cpu().numpy() - ref_gw) <= 1e-5 * scale + 1e-6 * np.abs(ref_gw)).all()


@pytest.mark.parametrize("order", ["asc", "shuffled"])
def test_adjoint_short_gradient_long_delays(order):
    """A short output gradient under long delays: most (row tile, time tile)
    pairs have DM trials whose staged windows miss the gradient's samples
    entirely, and some tiles have none that meet them; the kernels skip
    those passes.  With DM trials in order the skipped passes sit at both
    ends of each tile; shuffled, only the ends that happen to be dead are.
    grad_in must still equal the oracle's gather bit for bit."""
    dd = _dd()
    rng = np.random.default_rng(23)
    nc, nd, ns = 256, 96, 300
    f = 1270 + (np.arange(nc) + 0.5) * 300 / nc
    dms = np.arange(nd) * 2.0
    if order == "shuffled":
        dms = rng.permutation(dms)
    delta = oracle.delay_table(f, 5e-5, dms)
    nin = ns + int(delta.max())
    assert nin > 2 * 1280  # several time tiles, most of them far from the gradient's samples
    g = rng.standard_normal((1, nd, ns)).astype(np.float32)
    x = rng.standard_normal((1, nc, nin)).astype(np.float32)
    ref = oracle.adjoint_gather_f32(g, delta, nin)
    ref_gw, scale = oracle.grad_w(x, g, delta)
    plan = dd.Plan(f, 5e-5, dms)
    for v in _adj_variants(plan):
        _note(f"adjoint short gradient {order} variant {v}")
        plan.set_adjoint_variant(v)
        gi, gw = dd.adjoint(_rows(g), plan, nin, None, _rows(x))
        torch.cuda.synchronize()
        assert np.array_equal(gi.cpu().numpy(), ref), (order, v)
        assert (np.abs(gw.cpu().numpy() - ref_gw) <= 1e-5 * scale + 1e-6 * np.abs(ref_gw)).all(), (order, v)


def test_adjoint_dot_identity_config4_geometry():
    """<A x, g> == <x, A^T g> on one beam of the differentiable workload's geometry."""
    dd = _dd()
    b = synth.config(4)[0]
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + plan.max_delay
    _note(f"config4 geometry nin={nin}, adjoint variant {plan.adjoint_variant()}")
    torch.manual_seed(0)
    x = _rows(np.zeros((1, b.nchan, nin), np.float32))
    x.copy_(torch.randint(-4, 5, x.shape, device="cuda").float())
    g = _rows(np.zeros((1, b.ndm, b.nsamp), np.float32))
    g.copy_(torch.randint(-4, 5, g.shape, device="cuda").float())
    y = dd.dedisperse(x, plan, nsamp=b.nsamp)
    gi, _ = dd.adjoint(g, plan, nin)
    torch.cuda.synchronize()
    lhs = float((y.double() * g.double()).sum())
    rhs = float((x.double() * gi.double()).sum())
    assert lhs == rhs  # small integers: every sum is exact


def test_adjoint_config4_full_size_sampled():
    """The differentiable workload at full size (32 beams, 1024 channels, 1024
    DMs, 20,000 samples) in the adjoint launch the benchmark times: grad_in
    bit for bit on 6 channels of 2 beams, grad_w on those 6 channels (summed
    over all 32 beams) within 1e-5 of sum |g * x|."""
    dd = _dd()
    beams = synth.config(4)
    b = beams[0]
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + plan.max_delay
    nb = len(beams)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(404)
    x = _rows(np.zeros((nb, b.nchan, nin), np.float32))
    x.copy_(torch.randn(x.shape, generator=gen, device="cuda"))
    g = _rows(np.zeros((nb, b.ndm, b.nsamp), np.float32))
    g.copy_(torch.randn(g.shape, generator=gen, device="cuda"))
    w = torch.rand(b.nchan, generator=gen, device="cuda") + 0.5
    _note(f"config4 full size: adjoint variant {plan.adjoint_variant()}")
    gi, gw = dd.adjoint(g, plan, nin, w, x)
    torch.cuda.synchronize()
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    chans = np.array([0, 1, 333, 511, 900, b.nchan - 1])
    wn = w.cpu().numpy()
    gn = np.ascontiguousarray(g.cpu().numpy())
    for bi in (0, nb - 1):
        ref = oracle.adjoint_gather_f32(gn[bi:bi + 1], np.ascontiguousarray(delta[:, chans]), nin, wn[chans])
        got = gi[bi, chans].cpu().numpy()
        assert np.array_equal(got, ref[0]), f"grad_in beam {bi}"
    xs = np.ascontiguousarray(x[:, chans].cpu().numpy())
    ref_gw, scale = oracle.grad_w(xs, gn, np.ascontiguousarray(delta[:, chans]))
    got_gw = gw.cpu().numpy()[chans].astype(np.float64)
    assert (np.abs(got_gw - ref_gw) <= 1e-5 * scale + 1e-6 * np.abs(ref_gw)).all()


def _snr_t(y):
    return (y.max() - y.mean()) / y.std(correction=0)


def test_autograd_against_oracle_and_fd():
    dd = _dd()
    b = synth.config(0)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    ns = 1024
    nin = ns + int(delta.max())
    rng = np.random.default_rng(23)
    x = rng.standard_normal((1, b.nchan, nin)).astype(np.float32)
    synth.inject(x[0], delta, 17, 300, 4, 5.0)
    w = rng.uniform(0.8, 1.2, b.nchan).astype(np.float32)
    picks = [(0, 17), (0, 4)]
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    xg = _rows(x).requires_grad_(True)
    wg = torch.from_numpy(w).cuda().requires_grad_(True)
    out = dd.dedisperse_autograd(xg, plan, wg, ns)
    loss = -torch.stack([_snr_t(out[bb, j]) for bb, j in picks]).mean()
    loss.backward()
    torch.cuda.synchronize()
    gx = xg.grad.cpu().numpy().astype(np.float64)
    gw = wg.grad.cpu().numpy().astype(np.float64)
    # oracle FP64 chain: snr gradient -> adjoint -> (w * G, sum x * G)
    x64, w64 = x.astype(np.float64), w.astype(np.float64)
    o64 = oracle.forward_f64(x64, delta, ns, w64)
    g = np.zeros_like(o64)
    for bb, j in picks:
        g[bb, j] -= oracle.snr_grad(o64[bb, j]) / len(picks)
    G = oracle.adjoint_gather_f64(g, delta, nin)[0]
    ref_gw = (x64 * G).sum(axis=(0, 2))
    ref_gx = w64[None, :, None] * G
    assert np.allclose(gw, ref_gw, rtol=2e-4, atol=2e-5 * np.abs(ref_gw).max())
    assert np.allclose(gx, ref_gx, rtol=2e-4, atol=2e-5 * np.abs(ref_gx).max())

    # central finite differences of the FP64 oracle loss
    def L(xv, wv):
        return oracle.snr_loss(oracle.forward_f64(xv, delta, ns, wv), picks)

    eps = 1e-3
    for c in range(0, b.nchan, 9):
        e = np.zeros(b.nchan)
        e[c] = eps
        fd = (L(x64, w64 + e) - L(x64, w64 - e)) / (2 * eps)
        assert abs(fd - gw[c]) <= 1e-3 * max(1e-2, abs(fd)), (c, fd, gw[c])
    for (c, t) in [(0, 300 + int(delta[17, 0])), (63, 301), (20, 500)]:
        e = np.zeros_like(x64)
        e[0, c, t] = eps
        fd = (L(x64 + e, w64) - L(x64 - e, w64)) / (2 * eps)
        assert abs(fd - gx[0, c, t]) <= 1e-3 * max(1e-3, abs(fd)), (c, t, fd, gx[0, c, t])


def test_adjoint_autotune_keeps_a_correct_variant():
    dd = _dd()
    b = synth.config(0)[0]
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    times = plan.autotune_adjoint(2, b.nsamp)
    _note(f"adjoint autotune: {times}")
    assert "direct" in times and len(times) >= 3
    chosen = plan.adjoint_variant()
    names = dd.variant_names("f32")
    best = min(times, key=times.get)
    assert (best == "direct" and chosen == -1) or names[chosen] == best
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    rng = np.random.default_rng(23)
    g = rng.standard_normal((2, b.ndm, b.nsamp)).astype(np.float32)
    gi, _ = dd.adjoint(_rows(g), plan, nin)
    torch.cuda.synchronize()
    assert np.array_equal(gi.cpu().numpy(), oracle.adjoint_gather_f32(g, delta, nin))
