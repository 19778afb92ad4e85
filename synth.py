"""Seeded synthetic workloads for brute-force dedispersion.

This module only draws inputs: observing set-ups (channel frequencies, sample
time, DM trial lists), seeded noise, uint8 quantisation, the positions of
injected pulses and synthetic RFI channels.  It holds none of the method's
arithmetic: where a dispersed pulse is injected, the caller passes the integer
delay table to use.  Both the CPU oracle side and the GPU side draw their
inputs from here.

Set-ups follow the two survey scenarios of the paper (Section 3, Table 2:
LOFAR-like with 32 channels at 200,000 samples/s, Apertif-like with 1,024
channels at 20,000 samples/s; DM trials starting at 0) with the band edges,
DM steps and sizes of the workloads below.  Channel frequencies are the
centres of equal sub-bands, ascending.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 1601


@dataclass
class Beam:
    """One beam of one workload: observing set-up and input recipe."""

    nchan: int
    lo_mhz: float
    hi_mhz: float
    tsamp_s: float
    nsamp: int  # output samples per DM trial
    ndm: int
    dm_step: float
    dtype: str  # "f32" or "u8"
    seed: int
    npulse: int = 0
    pulse_width: int = 4
    pulse_amp: float = 1.0
    pulse_dm_index: list = field(default_factory=list)  # fixed pulse DMs (else drawn)
    pulse_t0: list = field(default_factory=list)

    def freqs(self) -> np.ndarray:
        c = np.arange(self.nchan, dtype=np.float64)
        return self.lo_mhz + (c + 0.5) * (self.hi_mhz - self.lo_mhz) / self.nchan

    def dms(self) -> np.ndarray:
        return np.arange(self.ndm, dtype=np.float64) * self.dm_step

    def elem_bytes(self) -> int:
        return 1 if self.dtype == "u8" else 4


def padded_len(n: int, elem_bytes: int, align_bytes: int = 16) -> int:
    """Smallest row length >= n whose byte size is a multiple of align_bytes."""
    q = align_bytes // elem_bytes
    return (n + q - 1) // q * q


def config(k: int) -> list[Beam]:
    """The five workloads, as lists of beams."""
    s = SEED_BASE + k
    if k == 0:
        # Tiny: 64 ch over 1400-1500 MHz, 50 us, 4096 samples, DMs 0..31 step 1,
        # one boxcar pulse (width 4, amplitude 5) at DM 17.
        return [Beam(64, 1400.0, 1500.0, 50e-6, 4096, 32, 1.0, "f32", s, npulse=1, pulse_width=4,
                     pulse_amp=5.0, pulse_dm_index=[17], pulse_t0=[2048])]
    if k == 1:
        # Apertif-like: 1024 ch over 1270-1570 MHz, 50 us, 20,000 samples,
        # 2048 DMs step 0.25, 8 pulses (width 4, amplitude 1).
        return [Beam(1024, 1270.0, 1570.0, 50e-6, 20000, 2048, 0.25, "f32", s, npulse=8)]
    if k == 2:
        # LOFAR-like: 32 ch over 6.25 MHz centred at 138 MHz, 5 us,
        # 200,000 samples, 2048 DMs step 0.01, uint8 input.
        return [Beam(32, 138.0 - 3.125, 138.0 + 3.125, 5e-6, 200000, 2048, 0.01, "u8", s)]
    if k == 3:
        # 256 uneven beams: channels from {256,512,1024,1536}, DMs U[512,4096]
        # step 0.25, samples U[8000,20000], 1270-1570 MHz, 50 us, 2 pulses each.
        rng = np.random.default_rng(s)
        beams = []
        for b in range(256):
            nc = int(rng.choice([256, 512, 1024, 1536]))
            nd = int(rng.integers(512, 4096, endpoint=True))
            ns = int(rng.integers(8000, 20000, endpoint=True))
            beams.append(Beam(nc, 1270.0, 1570.0, 50e-6, ns, nd, 0.25, "f32", s * 1000 + b, npulse=2))
        return beams
    if k == 4:
        # Differentiable: 32 Apertif-like beams, 1024 ch, 1024 DMs, 20,000
        # samples, one pulse per beam; RFI channels are drawn by rfi_channels().
        return [Beam(1024, 1270.0, 1570.0, 50e-6, 20000, 1024, 0.25, "f32", s * 1000 + b, npulse=1)
                for b in range(32)]
    raise ValueError(f"no workload {k}")


def pulses(beam: Beam, max_delay: int) -> list[tuple[int, int]]:
    """(dm index, start sample) of each pulse of a beam, drawn by its seed."""
    if beam.pulse_dm_index:
        return list(zip(beam.pulse_dm_index, beam.pulse_t0))
    rng = np.random.default_rng([beam.seed, 7])
    js = rng.integers(0, beam.ndm, size=beam.npulse)
    ts = rng.integers(0, beam.nsamp - beam.pulse_width, size=beam.npulse, endpoint=True)
    return [(int(j), int(t)) for j, t in zip(js, ts)]


def noise(beam: Beam, nin: int, stride: int | None = None) -> np.ndarray:
    """Seeded noise of shape [nchan][stride]; samples past nin are zero.

    f32: N(0, 1).  u8: clip(rint(128 + 16 N(0, 1)), 0, 255).
    """
    stride = nin if stride is None else stride
    rng = np.random.default_rng(beam.seed)
    if beam.dtype == "u8":
        x = np.zeros((beam.nchan, stride), np.uint8)
        for c in range(beam.nchan):
            v = rng.standard_normal(nin, dtype=np.float32)
            x[c, :nin] = np.clip(np.rint(128.0 + 16.0 * v), 0, 255).astype(np.uint8)
        return x
    x = np.zeros((beam.nchan, stride), np.float32)
    for c in range(beam.nchan):
        x[c, :nin] = rng.standard_normal(nin, dtype=np.float32)
    return x


def inject(x: np.ndarray, delay: np.ndarray, j: int, t0: int, width: int, amp: float) -> None:
    """Add a boxcar pulse of the given width and amplitude, dispersed along
    the supplied delay row: x[c][t0 + delay[j][c] + k] += amp for k < width."""
    for c in range(x.shape[0]):
        s = t0 + int(delay[j, c])
        x[c, s:s + width] += np.asarray(amp, dtype=x.dtype)


def rfi_channels(nchan: int, seed: int, frac: float = 0.05) -> np.ndarray:
    """Sorted indices of floor(frac * nchan) channels chosen by seed."""
    n = int(np.floor(frac * nchan))
    rng = np.random.default_rng([seed, 11])
    return np.sort(rng.choice(nchan, size=n, replace=False))


def add_rfi(x: np.ndarray, chans: np.ndarray, seed: int, sigma: float = 10.0) -> None:
    """Add seeded N(0, sigma^2) noise to the listed channels (synthetic RFI)."""
    rng = np.random.default_rng([seed, 13])
    nin = x.shape[1]
    for c in chans:
        x[c] += (sigma * rng.standard_normal(nin, dtype=np.float32)).astype(x.dtype)


def small_ints(rng: np.random.Generator, shape, lo=-8, hi=8, dtype=np.float32) -> np.ndarray:
    """Small integers as floats: every sum in the tests stays exact in FP32."""
    return rng.integers(lo, hi, size=shape, endpoint=True).astype(dtype)
