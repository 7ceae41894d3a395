"""Host-side logic of bench.py (no GPU): the traffic figure is reported only
for the kernel sources its counters were taken on, and only one GPU is
accepted."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write(tmp_path, sha):
    t = {"calibration": {"FETCH_SIZE": 2.0, "WRITE_SIZE": 1.0},
         "kernel_sources_sha256": sha,
         "workloads": {"9_80": {"kernels": {"k_scatter_rec": {
             "launches": 21, "fetch_kib_per_launch": 100.0, "write_kib_per_launch": 300.0}}}}}
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(t))
    return str(p)


def test_traffic_is_calibrated_bytes_per_launch(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC", _write(tmp_path, bench.kernel_sources_sha256()))
    assert bench.measured_traffic("9_80", "k_scatter_rec") == (100.0 * 2.0 + 300.0 * 1.0) * 1024
    assert bench.measured_traffic("9_80", "k_join_grouped") is None      # not counted
    assert bench.measured_traffic("10_90s", "k_scatter_rec") is None     # no such run


def test_traffic_is_dropped_once_the_kernels_change(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC", _write(tmp_path, "0" * 64))
    assert bench.measured_traffic("9_80", "k_scatter_rec") is None
    monkeypatch.setattr(bench, "TRAFFIC", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("9_80", "k_scatter_rec") is None


def test_kernel_hash_covers_the_kernel_sources(tmp_path, monkeypatch):
    h = bench.kernel_sources_sha256()
    for f in bench.KERNEL_SOURCES:
        src = os.path.join(ROOT, f)
        assert os.path.isfile(src)
        copy = tmp_path / os.path.basename(f)
        copy.write_bytes(open(src, "rb").read() + b"\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", tuple(os.path.basename(f) for f in bench.KERNEL_SOURCES))
    assert bench.kernel_sources_sha256() != h


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
