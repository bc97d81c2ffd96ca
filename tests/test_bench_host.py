"""Host-side logic of bench.py (no GPU): the one-GPU contract, the byte
counts behind the roofline figures, and the traffic lookup's source check."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_attraction_bytes(bench):
    # per nonzero a column word and a value; per row its offset, z_i, z_j and A_i
    assert bench.attract_bytes(10, 100, 4) == 100 * 8 + 10 * (8 + 24)
    assert bench.attract_bytes(10, 100, 8) == 100 * 12 + 10 * (8 + 48)
    # the benchmark's size (n = 1M, nnz = 257,760,766, FP32): 2.094 GB
    assert abs(bench.attract_bytes(1_000_000, 257_760_766, 4) - 2.094086128e9) < 1


def test_tree_bytes(bench):
    assert bench.tree_bytes(10, 7, 4) == 10 * (16 + 32 + 8) + 7 * 20


def _write_traffic(path, sources):
    entry = {"sources_sha256": sources, "fetch_kib": 1000.0, "write_kib": 10.0,
             "fetch_scale": 2.0, "write_scale": 1.0}
    with open(path, "w") as f:
        json.dump({"kernels": {"k": entry}}, f)


def test_traffic_lookup_follows_its_sources(bench, tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("first version\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    traffic = tmp_path / "traffic.json"
    _write_traffic(traffic, {str(src): sha})
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(traffic))
    assert bench.measured_traffic("k") == (1000.0 * 2.0 + 10.0) * 1024
    assert bench.measured_traffic("other") is None
    # a changed source invalidates the figure
    src.write_text("second version\n")
    assert bench.measured_traffic("k") is None
    # a missing source, or a missing summary, too
    _write_traffic(traffic, {str(tmp_path / "gone.hip"): sha})
    assert bench.measured_traffic("k") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.json"))
    assert bench.measured_traffic("k") is None


def test_committed_traffic_summary_is_well_formed(bench):
    with open(bench.TRAFFIC_FILE) as f:
        d = json.load(f)
    assert d["calibration"]["copy_bytes"] == 1 << 30
    for name, e in d["kernels"].items():
        assert set(e) >= {"sources_sha256", "fetch_kib", "write_kib", "fetch_scale",
                          "write_scale"}, name
        for path in e["sources_sha256"]:
            assert os.path.exists(os.path.join(ROOT, path)), path
