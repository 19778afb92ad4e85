"""GPU checks of the allocation-free adjoint (dedisp_adjoint_noalloc) against
the adjoint with a caller workspace (dedisp_adjoint), both called through the
C-ABI: grad_in and grad_w bit-identical, on two calls in a row with the second
smaller, for the tiled and the direct kernel; grad_in also bit-identical to
the oracle's gather and grad_w within 1e-5 of sum |g * x| of its FP64
definition.  Refusals (unprepared plan, partial sums larger than the fixed
scratch) are host-side checks that launch nothing.
"""
import ctypes

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


def _rows(x):
    dd = _dd()
    t = dd.empty_rows(x.shape[0], x.shape[1], x.shape[2], torch.float32, "cuda", zero=True)
    t.copy_(torch.from_numpy(np.ascontiguousarray(x)))
    return t


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _with_workspace(plan, g, nsamp, nin, w, x, gi, gw):
    """dedisp_adjoint with a workspace of the size it asks for."""
    dd = _dd()
    nb = g.shape[0]
    nbytes = dd.lib().dedisp_adjoint_workspace_bytes(plan.handle, nb, nin)
    ws = torch.empty(max(nbytes, 8), dtype=torch.uint8, device="cuda")
    st = dd.lib().dedisp_adjoint(plan.handle, nb, nsamp, nin, _p(g), g.stride(1), _p(w), _p(x), x.stride(1), _p(gi),
                                 gi.stride(1), _p(gw), _p(ws), nbytes, None)
    assert st == 0, dd.lib().dedisp_last_error()
    torch.cuda.synchronize()


def _noalloc(plan, g, nsamp, nin, w, x, gi, gw):
    dd = _dd()
    st = dd.lib().dedisp_adjoint_noalloc(plan.handle, g.shape[0], nsamp, nin, _p(g), g.stride(1), _p(w), _p(x),
                                         x.stride(1), _p(gi), gi.stride(1), _p(gw), None)
    assert st == 0, dd.lib().dedisp_last_error()
    torch.cuda.synchronize()


@pytest.mark.parametrize("variant", ["default", "direct"])
def test_noalloc_adjoint_matches_workspace_adjoint(variant):
    dd = _dd()
    b = synth.config(0)[0]
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    if variant == "direct":
        plan.set_adjoint_variant(-1)
    plan.prepare("f32", adjoint=True)
    delta = plan.delays()
    rng = np.random.default_rng(31)
    w = torch.from_numpy(rng.uniform(0.5, 1.5, b.nchan).astype(np.float32)).cuda()
    # two calls in a row, the second with fewer beams and samples: the shared
    # scratch keeps the first call's partial sums, which must not leak in
    for nb, ns in ((3, b.nsamp), (1, b.nsamp // 2 + 7)):
        nin = ns + int(delta.max()) + 5
        _note(f"noalloc adjoint ({variant}): {nb} beams, {ns} samples, nin {nin}")
        gh = rng.standard_normal((nb, b.ndm, ns)).astype(np.float32)
        xh = rng.standard_normal((nb, b.nchan, nin)).astype(np.float32)
        g, x = _rows(gh), _rows(xh)
        gi_ref = dd.empty_rows(nb, b.nchan, nin, torch.float32, "cuda")
        gw_ref = torch.empty(b.nchan, dtype=torch.float32, device="cuda")
        gi = dd.empty_rows(nb, b.nchan, nin, torch.float32, "cuda")
        gw = torch.full((b.nchan,), float("nan"), dtype=torch.float32, device="cuda")
        assert 0 < dd.lib().dedisp_adjoint_noalloc_bytes(plan.handle, nb, nin) <= 8 << 20
        _with_workspace(plan, g, ns, nin, w, x, gi_ref, gw_ref)
        _noalloc(plan, g, ns, nin, w, x, gi, gw)
        gi_h, gw_h = gi.cpu().numpy(), gw.cpu().numpy()
        assert np.array_equal(gi_h, gi_ref.cpu().numpy())
        assert np.array_equal(gw_h, gw_ref.cpu().numpy())
        # and the oracle: the gather form bit for bit, grad_w from its FP64 definition
        wh = w.cpu().numpy()
        want = oracle.adjoint_gather_f32(gh, delta, nin, wh)
        assert np.array_equal(gi_h, want)
        gw_def, scale = oracle.grad_w(xh, gh, delta)
        assert (np.abs(gw_h.astype(np.float64) - gw_def) <= 1e-5 * scale).all()


def test_noalloc_adjoint_refusals():
    dd = _dd()
    lib = dd.lib()
    b = synth.config(0)[0]
    plan = dd.Plan(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + plan.max_delay
    g = dd.empty_rows(1, b.ndm, b.nsamp, torch.float32, "cuda", zero=True)
    x = dd.empty_rows(1, b.nchan, nin, torch.float32, "cuda", zero=True)
    gi = dd.empty_rows(1, b.nchan, nin, torch.float32, "cuda")
    gw = torch.empty(b.nchan, dtype=torch.float32, device="cuda")
    # the adjoint kernel is not chosen yet: choosing it would build tables
    assert lib.dedisp_adjoint_noalloc_bytes(plan.handle, 1, nin) == 0
    st = lib.dedisp_adjoint_noalloc(plan.handle, 1, b.nsamp, nin, _p(g), g.stride(1), None, _p(x), x.stride(1),
                                    _p(gi), gi.stride(1), _p(gw), None)
    assert st == 1 and b"prepare" in lib.dedisp_last_error()
    plan.prepare("f32", adjoint=True)
    _noalloc(plan, g, b.nsamp, nin, None, x, gi, gw)
    # partial sums larger than the fixed scratch: refused before any launch
    # (every buffer really has the size of the call)
    cap = 8 << 20
    assert lib.dedisp_adjoint_noalloc_bytes(plan.handle, 1, nin) > 0
    nb = 1
    while lib.dedisp_adjoint_noalloc_bytes(plan.handle, nb, nin) <= cap:
        nb *= 2
    _note(f"noalloc adjoint refusal: {nb} beams need "
          f"{lib.dedisp_adjoint_noalloc_bytes(plan.handle, nb, nin)} bytes > {cap}")
    gbig = dd.empty_rows(nb, b.ndm, b.nsamp, torch.float32, "cuda", zero=True)
    xbig = dd.empty_rows(nb, b.nchan, nin, torch.float32, "cuda", zero=True)
    gibig = dd.empty_rows(nb, b.nchan, nin, torch.float32, "cuda")
    st = lib.dedisp_adjoint_noalloc(plan.handle, nb, b.nsamp, nin, _p(gbig), gbig.stride(1), None, _p(xbig),
                                    xbig.stride(1), _p(gibig), gibig.stride(1), _p(gw), None)
    assert st == 8 and b"scratch" in lib.dedisp_last_error()  # DEDISP_E_WORKSPACE
    # without the weight gradient the scratch is not used, so the size does not matter
    st = lib.dedisp_adjoint_noalloc(plan.handle, nb, b.nsamp, nin, _p(gbig), gbig.stride(1), None, None, 0,
                                    _p(gibig), gibig.stride(1), None, None)
    assert st == 0, lib.dedisp_last_error()
    torch.cuda.synchronize()
