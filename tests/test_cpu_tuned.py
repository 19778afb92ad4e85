"""The tuned multi-core CPU comparator (the paper's CPU implementation,
Section 5) against the oracle: it keeps Algorithm 1's per-output channel
order, so FP32 results must be bit-identical and uint8 sums exact, for every
tile configuration; invalid arguments are rejected."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def cpu():
    from paper_1601_01165_amd import cpu as c

    if not os.path.exists(c.LIB):
        c.build()
    return c


def test_exports_every_declared_symbol(cpu):
    text = open(os.path.join(ROOT, "include", "dedisp_cpu.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(ddcpu_[a-z0-9_]+)\s*\(", text))
    assert len(names) >= 6
    lib = ctypes.CDLL(cpu.LIB)
    for n in names:
        assert hasattr(lib, n), n


def test_config0_every_config_bit_identical(cpu):
    b = synth.config(0)[0]
    delta = oracle.delay_table(b.freqs(), b.tsamp_s, b.dms())
    nin = b.nsamp + int(delta.max())
    x = synth.noise(b, nin)
    for j, t0 in synth.pulses(b, int(delta.max())):
        synth.inject(x, delta, j, t0, b.pulse_width, b.pulse_amp)
    ref = oracle.forward_f32(x[None], delta, b.nsamp)
    w = np.random.default_rng(3).uniform(0.25, 2.0, b.nchan).astype(np.float32)
    refw = oracle.forward_f32(x[None], delta, b.nsamp, w)
    for i in range(len(cpu.configs())):
        assert np.array_equal(cpu.forward(x[None], delta, b.nsamp, cfg=i), ref), i
        assert np.array_equal(cpu.forward(x[None], delta, b.nsamp, w, cfg=i), refw), i


@pytest.mark.parametrize("shape", [(1, 1, 1, 1), (3, 5, 7, 2), (17, 70, 300, 1), (40, 9, 1031, 3)])
def test_ragged_f32_and_u8(cpu, shape):
    nc, nd, ns, nb = shape
    rng = np.random.default_rng(nc * 31 + nd)
    f = 1270.0 + (np.arange(nc) + 0.5) * 300.0 / nc
    dms = rng.permutation(np.arange(nd) * 0.5)
    delta = oracle.delay_table(f, 5e-5, dms)
    nin = ns + int(delta.max()) + 3
    x = rng.standard_normal((nb, nc, nin)).astype(np.float32)
    xu = rng.integers(0, 256, (nb, nc, nin)).astype(np.uint8)
    ref = oracle.forward_f32(x, delta, ns)
    refu = oracle.forward_u8(xu, delta, ns)
    for i in range(len(cpu.configs())):
        assert np.array_equal(cpu.forward(x, delta, ns, cfg=i), ref), (shape, i)
        assert np.array_equal(cpu.forward(xu, delta, ns, cfg=i), refu), (shape, i)


def test_rejects_invalid(cpu):
    lib = cpu.lib()
    x = np.zeros((1, 4, 100), np.float32)
    d = np.zeros((2, 4), np.int32)
    out = np.zeros((1, 2, 50), np.float32)
    ok = lib.ddcpu_forward_f32(1, 4, 2, 50, x.ctypes.data, 100, d.ctypes.data, None, out.ctypes.data, 50, 0)
    assert ok == 0
    assert lib.ddcpu_forward_f32(1, 4, 2, 50, None, 100, d.ctypes.data, None, out.ctypes.data, 50, 0) == 1
    assert lib.ddcpu_forward_f32(1, 4, 2, 50, x.ctypes.data, 100, d.ctypes.data, None, out.ctypes.data, 50, 99) == 1
    d[1, 2] = 60  # in_stride 100 < 50 + 60
    assert lib.ddcpu_forward_f32(1, 4, 2, 50, x.ctypes.data, 100, d.ctypes.data, None, out.ctypes.data, 50, 0) == 1
    d[1, 2] = -1
    assert lib.ddcpu_forward_f32(1, 4, 2, 50, x.ctypes.data, 100, d.ctypes.data, None, out.ctypes.data, 50, 0) == 1
    assert cpu.isa() in ("avx512f", "avx2", "generic")
    assert cpu.num_threads() >= 1
