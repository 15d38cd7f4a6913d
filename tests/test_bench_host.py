"""Host-side logic of the benchmark script: stored HBM-counter lookups and
the single-GPU contract (no GPU needed)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _records():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        return json.load(fh)


def test_traffic_lookup_matches_configuration_and_source(monkeypatch):
    recs = _records()
    assert recs
    for r in recs:
        monkeypatch.setattr(bench, "kernel_source_hash", lambda r=r: r["source"])
        assert bench.measured_traffic(r["workload"], r["precision"], r["rk"]) == r
        # counters of the monatomic gas never stand in for the (F, G) pair
        assert bench.measured_traffic(r["workload"], r["precision"], r["rk"], 2.0) is None
        # nor for another precision / scheme pair without its own record
        other = [x for x in recs if x["precision"] == 1 - r["precision"] and x["rk"] == r["rk"]]
        if not other:
            assert bench.measured_traffic(r["workload"], 1 - r["precision"], r["rk"]) is None
        # a changed kernel source invalidates the stored counters
        monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
        assert bench.measured_traffic(r["workload"], r["precision"], r["rk"]) is None


def test_traffic_records_are_at_least_algorithmic():
    # counted HBM bytes below the bytes the stage must move would mean a
    # miscalibrated counter scale
    for r in _records():
        assert r["bytes_per_launch"] >= 0.95 * r["algorithmic_bytes_per_launch"]


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode != 0
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]
