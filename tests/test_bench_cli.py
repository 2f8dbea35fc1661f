"""The benchmark's host-side contract, checked without a GPU: one GPU only, and the CPU
baseline record's fields (the oracle timed on a bounded sample of the same workload)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_cpu_baseline_record():
    sys.path.insert(0, ROOT)
    try:
        import bench
    finally:
        sys.path.remove(ROOT)
    rec = bench.cpu_baseline(0.01)
    assert rec["kind"] == "oracle" and rec["unit"] == "Msuffixes/s"
    assert rec["value"] > 0 and rec["cores"] >= 1
    assert "scale 0.01" in rec["sample"] and "SA+LCP+overlaps" in rec["sample"]
