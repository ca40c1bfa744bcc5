"""Host-side parts of bench.py: the one-GPU rule and the guard that drops
counted HBM traffic once a kernel source differs from the one it was counted
on.  No GPU is touched."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def test_traffic_guard(bench, tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_bytes(b"// kernel\n")
    import hashlib
    sha = hashlib.sha256(b"// kernel\n").hexdigest()[:16]
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    t = {"workload": "w", "bytes_per_launch": 1.5e6, "source": "kernel.hip",
         "sha256_prefix": sha}
    assert bench.counted_traffic(t, "w") == 1.5e6
    assert bench.counted_traffic(t, "other workload") is None
    src.write_bytes(b"// kernel, changed\n")
    assert bench.counted_traffic(t, "w") is None


def test_traffic_records_name_existing_sources_and_workloads(bench):
    for t in (bench.SPMM_TRAFFIC, bench.GRAM_TRAFFIC):
        assert os.path.isfile(os.path.join(ROOT, t["source"]))
        assert t["workload"] in bench.WORKLOADS
        assert len(t["sha256_prefix"]) == 16
