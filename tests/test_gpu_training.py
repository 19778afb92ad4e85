"""End-to-end training of per-channel weights through the adjoint.

The differentiable workload (Apertif-like beams with 5% of the channels
carrying high-variance synthetic RFI, a dispersed pulse per beam, loss = the
negative mean S/N at the pulse DMs) at a reduced size.  There is no paper
value for the outcome (parity unpinned); the checks are sanity properties:
the S/N improves over the run and the RFI channels end with smaller weights
than the clean ones.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _snr(y):
    return (y.max() - y.mean()) / y.std(correction=0)


def test_learned_rfi_weighting_improves_snr():
    import paper_1601_01165_amd as dd

    nb, nc, nd, ns = 4, 256, 128, 4096
    b0 = synth.Beam(nc, 1270.0, 1570.0, 50e-6, ns, nd, 0.25, "f32", 1605000, npulse=1)
    plan = dd.Plan(b0.freqs(), b0.tsamp_s, b0.dms())
    delta = plan.delays()
    nin = ns + plan.max_delay
    rfi = synth.rfi_channels(nc, 1605)
    x = np.zeros((nb, nc, nin), np.float32)
    picks = []
    for b in range(nb):
        beam = synth.Beam(nc, 1270.0, 1570.0, 50e-6, ns, nd, 0.25, "f32", 1605000 + b, npulse=1, pulse_amp=1.0)
        x[b] = synth.noise(beam, nin)
        synth.add_rfi(x[b], rfi, beam.seed)
        (j, t0), = synth.pulses(beam, plan.max_delay)
        synth.inject(x[b], delta, j, t0, beam.pulse_width, beam.pulse_amp)
        picks.append((b, j))
    xg = dd.empty_rows(nb, nc, nin, torch.float32, "cuda")
    xg.copy_(torch.from_numpy(x))
    w = torch.ones(nc, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([w], lr=0.05)
    hist = []
    for step in range(40):
        opt.zero_grad()
        out = dd.dedisperse_autograd(xg, plan, w, ns)
        loss = -torch.stack([_snr(out[b, j]) for b, j in picks]).mean()
        loss.backward()
        opt.step()
        hist.append(-float(loss))
    torch.cuda.synchronize()
    print(f"S/N: start {hist[0]:.2f}, end {hist[-1]:.2f}", flush=True)
    assert hist[-1] > 1.5 * hist[0]
    assert max(hist[-5:]) > max(hist[:5])
    wa = w.detach().abs().cpu().numpy()
    clean = np.setdiff1d(np.arange(nc), rfi)
    print(f"mean |w|: RFI {wa[rfi].mean():.3f}, clean {wa[clean].mean():.3f}", flush=True)
    assert wa[rfi].mean() < 0.5 * wa[clean].mean()
