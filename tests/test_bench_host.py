"""Host-side checks of the benchmark script (no GPU): the one-GPU rule, the host description, and the
lookup of stored HBM byte counters, which applies only to the kernel sources
they were measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_stored_traffic_matches_sources():
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    lines = [ln for ln in open(path) if ln.startswith("traffic ")]
    assert lines, "no traffic entries"
    h = bench.kernel_sources_hash()
    current = [dict(t.split("=", 1) for t in ln.split()[1:]) for ln in lines]
    for kv in current:
        if kv["sources"] == h:
            got = bench.stored_traffic(kv["workload"], kv["variant"])
            assert got == pytest.approx(float(kv["bytes_per_launch"]))
            assert got == pytest.approx(float(kv["fetch_bytes"]) + float(kv["write_bytes"]), rel=1e-5)
    assert bench.stored_traffic("lofar", "no-such-variant") is None


def test_stored_traffic_ignores_other_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "hbm_traffic.txt").write_text(
        "traffic workload=lofar variant=v1 sources=0000000000000000 bytes_per_launch=1e9 fetch_bytes=1 write_bytes=1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "ffffffffffffffff")
    assert bench.stored_traffic("lofar", "v1") is None
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "0000000000000000")
    assert bench.stored_traffic("lofar", "v1") == 1e9


def test_cpu_model_is_reported():
    host = bench.cpu_model()
    assert set(host) == {"model", "logical_cpus"}
    assert isinstance(host["model"], str) and host["model"]
    assert host["logical_cpus"] is None or host["logical_cpus"] >= 1
