#!/usr/bin/env python3
"""Benchmark: one step = the whole hot path on one large job -- validate/pack, suffix array by
prefix doubling over LSD radix sorts, Kasai LCP, and suffix-prefix overlaps by LCP-interval
walks -- over the plain large workload (5 Mbp genome, 100,000 reads of 500 bp, 0.5 %
substitutions, N = 50.1 M suffixes, overlaps >= 40), input resident in HBM.

Prints one JSON line.  `value` is suffixes per second of the whole step (Msuffixes/s); the
`roofline` object reports the radix pass kernel (the dominant kernel) from HIP events recorded
around each of its launches during the timed steps; `cpu_baseline` times the CPU oracle on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "SA build Msuffixes/s + % HBM peak; served jobs/s and p50/p99 vs plain path"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="plain-large-5M")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-scale", type=float, default=0.5)
    ap.add_argument("--digit-bits", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--items", type=int, default=0)
    ap.add_argument("--lcp-chunk", type=int, default=0)
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "radix_pass_traffic.json"),
                    help="JSON with HBM bytes per radix-pass launch from rocprofv3 counters")
    return ap.parse_args()


def cpu_baseline(scale):
    import oracle
    from paper_1404_3456_amd import synth
    r = synth.large_plain(scale=scale)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    t0 = time.perf_counter()
    sa = oracle.suffix_array(r.text, threads)
    lcp = oracle.lcp_array(r.text, sa, threads)
    ovl = oracle.overlaps(r.text, r.min_len, threads)
    dt = time.perf_counter() - t0
    return {
        "value": round(r.n / dt / 1e6, 4),
        "unit": "Msuffixes/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{r.name}: same recipe at scale {scale:g} (genome {r.genome_len} bp, "
                   f"{r.m} reads of 500 bp, 10x, 0.5% subs; N={r.n}); SA+LCP+overlaps "
                   f"({ovl.shape[0]} rows) in {dt:.2f} s"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                          "(the design for more GPUs is described, not run)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1404_3456_amd as pkg
    from paper_1404_3456_amd import synth

    pkg.load()
    if args.workload == "plain-large-5M":
        r = synth.large_plain()
    elif args.workload == "repeat-stress-40M":
        r = synth.repeat_stress()
    elif args.workload == "plain-small-20k":
        r = synth.small_plain()
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    tuning = None
    if args.digit_bits or args.block or args.items:
        tuning = pkg.Tuning(args.digit_bits, args.block, args.items, 0)
    if args.lcp_chunk:
        pkg.sa_lcp_set_chunk(args.lcp_chunk)
    log(f"workload {r.name}: n={r.n} m={r.m} sha256={r.sha256()[:16]}")
    dev = torch.device("cuda:0")
    text = torch.from_numpy(r.text).to(dev)
    n = r.n
    stream = torch.cuda.current_stream()

    def step():
        sa, isa = pkg.sa_build(text, tuning=tuning)
        lcp = pkg.sa_lcp(text, sa, isa)
        ovl = pkg.sa_overlaps(text, sa, isa, lcp, r.min_len)
        return sa, isa, lcp, ovl

    for i in range(args.warmup):
        out = step()
        torch.cuda.synchronize()
        log(f"warmup {i} done")
    pkg.sa_timing_reset()
    pkg.sa_timing_enable(True)
    sa_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sa, isa, rounds = pkg.sa_build(text, tuning=tuning, return_rounds=True)
        e1.record(stream)
        lcp = pkg.sa_lcp(text, sa, isa)
        ovl = pkg.sa_overlaps(text, sa, isa, lcp, r.min_len)
        torch.cuda.synchronize()
        sa_ms.append(e0.elapsed_time(e1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pkg.sa_timing_enable(False)
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step")

    kern = {}
    for key in ("radix_pass", "keybuild", "rank_update", "kasai", "overlap_walk", "pack"):
        L, ms, by = pkg.sa_timing_get(key)
        kern[key] = {"launches": L, "ms": round(ms, 4),
                     "avg_us": round(ms * 1000.0 / L, 3) if L else None,
                     "alg_GBs": round(by / (ms * 1e-3) / 1e9, 1) if ms > 0 else None}
    L, ms, by = pkg.sa_timing_get("radix_pass")
    achieved = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    traffic = None
    if os.path.exists(args.traffic):
        try:
            tr = json.load(open(args.traffic))
            traffic = tr.get("bytes_per_launch")
        except Exception:
            traffic = None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_onesweep (one LSD radix pass)",
                "alg_bytes_per_launch": round(by / L) if L else None,
                "avg_launch_us": round(ms * 1000.0 / L, 3) if L else None}

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(args.cpu_sample_scale)
        log(f"cpu baseline: {cpu['value']} Msuffixes/s on {cpu['cores']} threads")

    sa_build_ms = float(np.median(sa_ms))
    out = {
        "metric": METRIC,
        "value": round(n / (ms_per_step * 1e-3) / 1e6, 3),
        "unit": "Msuffixes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": r.name, "n_suffixes": n, "reads": r.m, "read_len": 500,
                   "genome_bp": r.genome_len, "substitution_rate": 0.005,
                   "min_overlap": r.min_len, "overlaps": int(ovl.shape[0]),
                   "sha256": r.sha256(), "tuning": tuning.__dict__ if tuning else "default"},
        "sa_build_ms": round(sa_build_ms, 3),
        "sa_build_Msuffixes_per_s": round(n / (sa_build_ms * 1e-3) / 1e6, 3),
        "sa_rounds": rounds,
        "kernels": kern,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
