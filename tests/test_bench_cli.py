"""The benchmark's host-side contract, checked without a GPU: one GPU only, the CPU baseline
record's fields (the oracle timed on bounded samples of the same workload, all threads and one
thread, stage by stage), the serving pool and the per-kernel byte figures."""
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
    rec = bench.cpu_baseline(0.01, 0.005)
    assert rec["kind"] == "oracle" and rec["unit"] == "Msuffixes/s"
    assert rec["value"] > 0 and rec["cores"] >= 1
    assert "scale 0.01" in rec["sample"] and "scale 0.005" in rec["sample"]
    allc, serial = rec["modes"]["all_cores"], rec["modes"]["single_thread"]
    assert allc["threads"] == rec["cores"] and serial["threads"] == 1
    for mode in (allc, serial):
        assert mode["sa_s"] > 0 and mode["lcp_s"] > 0 and mode["overlaps_s"] > 0
        assert mode["overlap_rows"] > 0
    assert rec["value"] == allc["Msuffixes_per_s"]
    assert rec["host"]["nproc"] >= 1


def test_serving_pool_matches_the_serial_generator():
    """The benchmark's parallel pool is the serving stream's first jobs, byte for byte."""
    sys.path.insert(0, ROOT)
    try:
        import bench
        from paper_1404_3456_amd import synth
    finally:
        sys.path.remove(ROOT)
    texts = bench.serving_pool(3)
    _, jobs = synth.serving_jobs(n_jobs=3, rate_per_s=1.0)
    assert [t.tobytes() for t in texts] == [j.text.tobytes() for j in jobs]


def test_survey_bytes_cover_the_build_kernels():
    sys.path.insert(0, ROOT)
    try:
        import bench
    finally:
        sys.path.remove(ROOT)
    for k in bench.BUILD_KEYS:
        assert bench.SURVEY_BYTES[k] > 0
    assert bench.SURVEY_BYTES["rank_update"] == 16.0 and bench.SURVEY_BYTES["kasai"] == 12.0
