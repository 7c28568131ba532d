"""CPU checks of the bench's host logic: one GPU only, and traffic figures
reported only when the committed counters were taken with the current kernel
sources."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def _traffic_file(tmp_path, sha):
    d = tmp_path / "profiles"
    d.mkdir()
    (d / "traffic.json").write_text(json.dumps({
        "kernels_sha1": sha,
        "entries": {"w/plain/vector_path": {"fetch_bytes": 1000, "write_bytes": 24}}}))


def test_traffic_needs_the_current_kernel_sources(tmp_path, monkeypatch):
    _traffic_file(tmp_path, "abc")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernels_sha1", lambda: "abc")
    assert bench.measured_traffic("w", "plain", "vector_path") == 1024
    assert bench.measured_traffic("w", "mixed", "vector_path") is None
    monkeypatch.setattr(bench, "kernels_sha1", lambda: "def")
    assert bench.measured_traffic("w", "plain", "vector_path") is None


def test_missing_or_damaged_traffic_file_gives_none(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w", "plain", "vector_path") is None
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text("{not json")
    assert bench.measured_traffic("w", "plain", "vector_path") is None


def test_committed_traffic_is_scaled_by_the_copy_calibration():
    """Every committed entry: bytes = counter KiB x 1024 x the copy kernel's
    scale (1 GiB read / what FETCH_SIZE reads for it, likewise for writes);
    on this device FETCH_SIZE counts half the bytes read and WRITE_SIZE all
    of those written, so the scales are about 2 and 1."""
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        t = json.load(f)
    sc = t["scale"]
    assert abs(sc["fetch"] - sc["copy_bytes"] / 1024 / sc["copy_kernel_fetch_kib"]) < 1e-5
    assert abs(sc["write"] - sc["copy_bytes"] / 1024 / sc["copy_kernel_write_kib"]) < 1e-5
    assert 1.99 < sc["fetch"] < 2.01 and 0.99 < sc["write"] < 1.01
    assert len(t["kernels_sha1"]) == 40 and t["entries"]
    for key, e in t["entries"].items():
        workload, mode, kernel = key.split("/")
        assert workload and mode in ("plain", "mixed") and kernel in ("vector_path", "window",
                                                                     "mfma_path")
        # the stored KiB (0.1) and scales (1e-6) are rounded; the bytes are not
        for kind in ("fetch", "write"):
            want = e[kind + "_kib_per_dispatch"] * 1024 * sc[kind]
            assert e[kind + "_bytes"] > 0 and abs(e[kind + "_bytes"] - want) <= 1e-6 * want + 1024
