#!/usr/bin/env python3
"""Benchmark: one step = the whole hot path on one large job -- validate/pack, suffix array by
prefix doubling over LSD radix sorts, Kasai LCP, and suffix-prefix overlaps by LCP-interval
walks -- over the plain large workload (5 Mbp genome, 100,000 reads of 500 bp, 0.5 %
substitutions, N = 50.1 M suffixes, overlaps >= 40), input resident in HBM.

Prints one JSON line.  `value` is suffixes per second of the whole step (Msuffixes/s); the
`roofline` object reports the kernel with the most time per step (the dominant kernel) from
HIP events recorded around each of its launches during the timed steps; `cpu_baseline` times
the CPU oracle on a bounded sample of the same workload.
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
    ap.add_argument("--seg-pack", type=int, default=0,
                    help="batched: at most this many characters per build (0: one build)")
    ap.add_argument("--sa-algo", choices=("doubling", "dc3"), default="doubling",
                    help="suffix-array construction of the timed path: prefix doubling "
                         "(sa_build) or the skew recursion (sa_build_dc3); same array")
    ap.add_argument("--max-total", type=int, default=0,
                    help="batched workload: stop adding sets once this many characters are drawn")
    ap.add_argument("--graph", action="store_true",
                    help="batched workload: replay the doubling rounds from a hipGraph (default: "
                         "host-driven rounds one ahead, measured faster)")
    ap.add_argument("--autotune", action="store_true",
                    help="choose digit width, tile shape (and, batched, set packing) by measurement first")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run sa_copy_u32 over 256 MiB three times (counter calibration)")
    ap.add_argument("--pool", type=int, default=64, help="serving: distinct jobs generated")
    ap.add_argument("--jobs", type=int, default=300, help="serving: jobs per arrival-rate run")
    ap.add_argument("--workers", type=int, default=4, help="serving: server worker streams")
    ap.add_argument("--max-jobs", type=int, default=64, help="serving: jobs per batch at most")
    ap.add_argument("--p99-bound-ms", type=float, default=500.0, help="serving: p99 bound")
    ap.add_argument("--patterns", type=int, default=1_000_000, help="lookup: patterns per step")
    ap.add_argument("--pattern-len", type=int, default=40, help="lookup: pattern length")
    ap.add_argument("--traffic-dir", default=os.path.join(ROOT, "profiles"),
                    help="folder of <kernel>_traffic.json files: HBM bytes per launch from rocprofv3 counters")
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


def bench_batched(args, pkg, torch, np):
    """256 independent fragment sets: one batched build (all sets per launch; doubling rounds
    driven from the host, or replayed from a hipGraph with --graph) against the plain path run
    set by set, same GPU, same stream."""
    from paper_1404_3456_amd import synth
    t0 = time.perf_counter()
    sets = synth.batched_sets(max_total=args.max_total or None)
    off = np.concatenate([[0], np.cumsum([s.text.size for s in sets])]).astype(np.int64)
    cat = np.concatenate([s.text for s in sets])
    log(f"batched workload: {len(sets)} sets, n={cat.size}, generated in {time.perf_counter()-t0:.1f} s")
    text = torch.from_numpy(cat).cuda()
    min_len = 40
    tuning = None
    if args.digit_bits or args.block or args.items or args.seg_pack:
        tuning = pkg.Tuning(args.digit_bits, args.block, args.items, args.seg_pack)
    tune_report = None
    if args.autotune:
        from paper_1404_3456_amd import autotune
        tuning, tune_report = autotune.autotune(
            text, off, candidates=[(8, 512, 16), (9, 512, 16), (9, 256, 16), (11, 512, 16)],
            seg_packs=(0, 1 << 28), reps=1, use_cache=False, log=log)
        log(f"autotuned: {tuning}")

    plain_tuning = None
    if tuning is not None and (tuning.digit_bits or tuning.block_threads or tuning.items_per_thread):
        plain_tuning = pkg.Tuning(tuning.digit_bits, tuning.block_threads, tuning.items_per_thread, 0)

    def batched():
        sa, isa = pkg.sa_build_batched(text, off, tuning=tuning, use_graph=args.graph)
        lcp = pkg.sa_lcp(text, sa, isa)
        ovl = pkg.sa_overlaps(text, sa, isa, lcp, min_len)
        return sa, ovl

    def plain():
        outs = []
        for s in range(len(sets)):
            t = text[off[s]:off[s + 1]]
            sa, isa = pkg.sa_build(t, tuning=plain_tuning)
            lcp = pkg.sa_lcp(t, sa, isa)
            outs.append(pkg.sa_overlaps(t, sa, isa, lcp, min_len))
        return outs

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            a = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - a
            best = dt if best is None else min(best, dt)
        return best, out

    tb, (sa_b, ovl_b) = timed(batched, args.steps)
    log(f"batched: {tb*1e3:.1f} ms")
    tp, outs = timed(plain, max(1, args.steps // 2))
    log(f"plain per set: {tp*1e3:.1f} ms")
    # the batched result must equal the per-set plain result (overlap rows per set)
    n_rows = sum(int(o.shape[0]) for o in outs)
    same = n_rows == int(ovl_b.shape[0])
    out = {
        "metric": "batched jobs/s vs plain per-job path",
        "value": round(len(sets) / tb, 3),
        "unit": "jobs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": round(tb * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "batched-256: 256 sets, genome log-uniform 10 kbp-2 Mbp, reads "
                               "100-1000 bp, coverage 5-20x, 0.5% subs, overlaps >= 40",
                   "sets": len(sets), "n_total": int(cat.size), "graph": args.graph,
                   "tuning": tuning.__dict__ if tuning else "default"},
        "plain_jobs_per_s": round(len(sets) / tp, 3),
        "speedup_vs_plain": round(tp / tb, 3),
        "batched_Msuffixes_per_s": round(cat.size / tb / 1e6, 1),
        "overlap_rows": int(ovl_b.shape[0]),
        "rows_match_plain": bool(same),
        "autotune": tune_report,
    }
    print(json.dumps(out), flush=True)


def bench_serving(args, pkg, torch, np):
    """Poisson stream of assembly jobs (genome log-uniform 1 kbp-5 Mbp, reads 150-800 bp, 8x,
    0.5% subs, overlaps >= 40), served by the continuous-batching server and, as the baseline,
    by the plain path (one job at a time, single-text entry points), both under a 64 GiB arena.
    Reports completed jobs/s and p50/p99 latency (completion minus scheduled arrival)."""
    import threading
    from paper_1404_3456_amd import synth
    t0 = time.perf_counter()
    pool_n = args.pool
    _, pool = synth.serving_jobs(n_jobs=pool_n, rate_per_s=1.0)
    texts = [j.text for j in pool]
    log(f"serving pool: {pool_n} jobs, {sum(t.size for t in texts)/1e6:.1f} M chars, "
        f"generated in {time.perf_counter()-t0:.1f} s")
    arena = 64 << 30

    def run(mode, rate, n_jobs, workers):
        # the same job sequence for every run; only the arrival times depend on the rate
        order = np.random.default_rng(1404).integers(0, pool_n, size=n_jobs)
        rng = np.random.default_rng(1404 + int(rate * 1000))
        gaps = rng.exponential(1.0 / rate, size=n_jobs) if rate > 0 else np.zeros(n_jobs)
        arr = np.cumsum(gaps) - gaps[0]
        lat = [None] * n_jobs
        pending = {}
        lock = threading.Lock()
        done = threading.Event()
        with pkg.AsmServer(arena, max_jobs_per_batch=args.max_jobs, workers=workers,
                           mode=mode) as srv:
            start = time.perf_counter()

            def submitter():
                for i in range(n_jobs):
                    target = start + arr[i]
                    while True:
                        now = time.perf_counter()
                        if now >= target:
                            break
                        time.sleep(min(0.0005, target - now))
                    lag = time.perf_counter() - target
                    jid = srv.asm_submit(texts[order[i]], 40, borrow=True)
                    with lock:
                        pending[jid] = (i, lag)
                done.set()

            th = threading.Thread(target=submitter)
            th.start()
            finished = 0
            t_last = start
            while finished < n_jobs:
                with lock:
                    items = list(pending.items())
                for jid, (i, lag) in items:
                    r = srv.asm_poll(jid)
                    if r is None:
                        continue
                    if r["status"] != 0:
                        raise RuntimeError(f"job failed with {r['status']}")
                    lat[i] = (r["t_done"] - r["t_submit"]) + lag
                    srv.asm_release(jid)
                    with lock:
                        del pending[jid]
                    finished += 1
                    t_last = time.perf_counter()
                if not items:
                    time.sleep(0.0002)
            th.join()
            stats = srv.asm_server_stats()
        lat = np.array(lat)
        span = t_last - start
        return {"rate": round(rate, 2), "jobs": n_jobs, "jobs_per_s": round(n_jobs / span, 2),
                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
                "batches": stats["batches"], "max_concurrent_batches": stats["max_concurrent_batches"]}

    # plain capacity: everything queued at once (closed loop, saturated)
    sat_p = run(1, 0.0, args.jobs, 1)
    mu_p = sat_p["jobs_per_s"]
    log(f"plain saturated: {sat_p}")
    sat_b = run(0, 0.0, args.jobs, args.workers)
    log(f"batched saturated: {sat_b}")
    curves = {"plain": [], "served": []}
    for k in (0.5, 1.0):
        curves["plain"].append(run(1, k * mu_p, args.jobs, 1))
        log(f"plain {k}x: {curves['plain'][-1]}")
    for k in (0.5, 1.0, 2.0, 3.0, 4.0, 6.0):
        curves["served"].append(run(0, k * mu_p, args.jobs, args.workers))
        log(f"served {k}x: {curves['served'][-1]}")
    bound_ms = args.p99_bound_ms
    ok = [c for c in curves["served"] if c["p99_ms"] <= bound_ms]
    best = max(ok, key=lambda c: c["jobs_per_s"]) if ok else None
    out = {
        "metric": "served jobs/s at p99 <= bound vs plain per-job path",
        "value": best["jobs_per_s"] if best else None,
        "unit": "jobs/s",
        "n_gpus": 1, "steps": args.jobs, "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "serving: Poisson jobs, genome log-uniform 1 kbp-5 Mbp, reads "
                               "150-800 bp, 8x, 0.5% subs, overlaps >= 40, 64 GiB arena",
                   "pool": pool_n, "jobs_per_run": args.jobs, "workers": args.workers,
                   "max_jobs_per_batch": args.max_jobs, "p99_bound_ms": bound_ms},
        "plain_capacity_jobs_per_s": mu_p,
        "served_saturated_jobs_per_s": sat_b["jobs_per_s"],
        "speedup_at_bound": round(best["jobs_per_s"] / mu_p, 3) if best else None,
        "saturated_speedup": round(sat_b["jobs_per_s"] / mu_p, 3),
        "best_point": best,
        "curves": curves,
    }
    print(json.dumps(out), flush=True)


def bench_lookup(args, pkg, torch, np):
    """Pattern lookup over the plain large workload's suffix array: one step = sa_lookup of
    `--patterns` seeded patterns of `--pattern-len` bases (substrings, read prefixes and random
    strings), patterns and suffix array resident in HBM."""
    from paper_1404_3456_amd import synth
    r = synth.large_plain()
    dev = torch.device("cuda:0")
    text = torch.from_numpy(r.text).to(dev)
    sa, _ = pkg.sa_build(text)
    L = args.pattern_len
    pats = synth.lookup_patterns(r.text, args.patterns, 0, L, L)
    off_h = np.zeros(len(pats) + 1, dtype=np.int64)
    off_h[1:] = np.cumsum([len(p) for p in pats])
    buf = torch.from_numpy(np.frombuffer(b"".join(pats), dtype=np.uint8).copy()).to(dev)
    off = torch.from_numpy(off_h).to(dev)
    log(f"lookup: n={r.n}, {len(pats)} patterns, {int(off_h[-1])} bases")
    for _ in range(args.warmup):
        pkg.sa_lookup(text, sa, (buf, off))
    torch.cuda.synchronize()
    pkg.sa_timing_reset()
    pkg.sa_timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = pkg.sa_lookup(text, sa, (buf, off))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pkg.sa_timing_enable(False)
    ms = (t1 - t0) * 1000.0 / args.steps
    Lk, kms, _ = pkg.sa_timing_get("lookup")
    res = res.cpu().numpy()
    found = int((res[:, 1] > res[:, 0]).sum())
    # modelled bytes per lookup: one joint search of ceil(log2 n) steps, plus for a pattern
    # that occurs cnt times the two searches inside its split interval (2 ceil(log2(cnt + 1))
    # steps); each step touches one 64-byte line of the suffix array and one of the text
    # records.  The kernel is bound by each thread's chain of dependent loads, not by this
    # traffic: the figure shows how far from the bandwidth roof that leaves it.
    cnt = (res[:, 1] - res[:, 0]).astype(np.int64)
    steps = int(np.ceil(np.log2(r.n))) * len(pats) + int(
        (2 * np.ceil(np.log2(cnt[cnt > 0] + 1))).sum())
    model = steps * 128.0
    kern_s = kms * 1e-3 / Lk
    print(json.dumps({
        "metric": "pattern lookups per second (SA interval of each pattern)",
        "value": round(len(pats) / (ms * 1e-3) / 1e6, 3), "unit": "Mlookups/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "lookup-plain-large-5M", "n_suffixes": r.n, "patterns": len(pats),
                   "pattern_len": L, "found": found},
        "kernel_ms": round(kern_s * 1e3, 4),
        "roofline": {"bound": "hbm", "achieved": round(model / kern_s / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(model / kern_s / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_lookup",
                     "model": "(ceil(log2 n) + 2*ceil(log2(count+1)) if found) steps x 128 B per lookup; latency-bound"},
    }), flush=True)


def bench_reconstruct(args, pkg, torch, np):
    """Cut-and-continue reconstruction: a 5 Mbp random sequence cut twice (cut positions at
    least 32 apart, ~500-base pieces, ~20,000 fragments, shuffled); one step = index build on
    the GPU (pack, SA, LCP), copy to the host, and the host search through the index."""
    from paper_1404_3456_amd import synth
    from paper_1404_3456_amd._abi import to_host
    text_h, seq, frags = synth.two_cuttings(0, 5_000_000, 500, min_gap=32)
    dev = torch.device("cuda:0")
    text = torch.from_numpy(text_h).to(dev)
    log(f"reconstruct: {len(frags)} fragments, n={text_h.size}")
    times = []
    for i in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sa, isa = pkg.sa_build(text)
        lcp = pkg.sa_lcp(text, sa, isa)
        sa_h, isa_h, lcp_h = to_host(sa, isa, lcp)
        t1 = time.perf_counter()
        res = pkg.sa_reconstruct_host(text_h, sa_h, isa_h, lcp_h)
        t2 = time.perf_counter()
        if i >= args.warmup:
            times.append((t1 - t0, t2 - t1))
    assert res is not None and res[0] == seq, "reconstruction differs from the sequence"
    idx = float(np.median([a for a, _ in times])) * 1e3
    srch = float(np.median([b for _, b in times])) * 1e3
    ms = idx + srch
    print(json.dumps({
        "metric": "fragments reconstructed per second (cut and continue through the SA)",
        "value": round(len(frags) / (ms * 1e-3), 1), "unit": "fragments/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "reconstruct-5Mbp-two-cuttings", "fragments": len(frags),
                   "n": int(text_h.size), "mean_fragment": 500, "min_gap": 32},
        "index_ms": round(idx, 3), "host_search_ms": round(srch, 3),
    }), flush=True)


def bench_overlaps_rc(args, pkg, torch, np):
    """Overlaps on both strands: 100,000 error-free reads of 500 bp from both strands of a
    5 Mbp genome (10x); one step = doubled text (reads + reverse complements, N = 100.2 M),
    SA, LCP, overlaps and strand naming, input resident in HBM."""
    from paper_1404_3456_amd import synth
    text_h, _, _ = synth.strand_reads(0, 5_000_000, 100_000, 500)
    dev = torch.device("cuda:0")
    text = torch.from_numpy(text_h).to(dev)
    for _ in range(args.warmup):
        pkg.sa_overlaps_rc(text, 40)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rows = pkg.sa_overlaps_rc(text, 40)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    n2 = 2 * text_h.size
    print(json.dumps({
        "metric": "both-strand overlap step, suffixes of the doubled text per second",
        "value": round(n2 / (ms * 1e-3) / 1e6, 3), "unit": "Msuffixes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "overlaps-rc-5Mbp-100k-reads", "n": int(text_h.size),
                   "n_doubled": int(n2), "reads": 100_000, "read_len": 500, "min_overlap": 40,
                   "rows": int(rows.shape[0]),
                   "rows_by_strand": [int((rows[:, 2] == k).sum().item()) for k in range(3)]},
    }), flush=True)


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
    if args.workload == "batched-256":
        return bench_batched(args, pkg, torch, np)
    if args.workload == "serving":
        return bench_serving(args, pkg, torch, np)
    if args.workload == "lookup":
        return bench_lookup(args, pkg, torch, np)
    if args.workload == "reconstruct":
        return bench_reconstruct(args, pkg, torch, np)
    if args.workload == "overlaps-rc":
        return bench_overlaps_rc(args, pkg, torch, np)
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
    if args.autotune:
        from paper_1404_3456_amd import autotune
        tuning, rep = autotune.autotune(text, reps=2, use_cache=False, log=log)
        log(f"autotuned: {tuning} ({rep['ms']} ms)")
    n = r.n
    stream = torch.cuda.current_stream()

    def build_sa():
        if args.sa_algo == "dc3":
            return pkg.sa_build_dc3(text, tuning=tuning, return_levels=True)
        return pkg.sa_build(text, tuning=tuning, return_rounds=True)

    def step():
        sa, isa, _ = build_sa()
        lcp = pkg.sa_lcp(text, sa, isa)
        ovl = pkg.sa_overlaps(text, sa, isa, lcp, r.min_len)
        return sa, isa, lcp, ovl

    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            pkg.sa_copy_u32(dst, src)
        torch.cuda.synchronize()
        log("calibration copy: 3 x 256 MiB read + 256 MiB written")
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
        sa, isa, rounds = build_sa()
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
    keys = ("radix_pass", "keybuild", "keyruns", "rank_update", "kasai", "overlap_walk", "pack")
    if args.sa_algo == "dc3":
        keys = ("radix_pass", "dc3_keys", "dc3_names", "dc3_lift", "dc3_recs", "dc3_merge", "kasai",
                "overlap_walk", "pack")
    for key in keys:
        L, ms, by = pkg.sa_timing_get(key)
        kern[key] = {"launches": L, "ms": round(ms, 4),
                     "avg_us": round(ms * 1000.0 / L, 3) if L else None,
                     "alg_GBs": round(by / (ms * 1e-3) / 1e9, 1) if ms > 0 else None}
    names = {"radix_pass": "k_onesweep (one LSD radix pass)",
             "rank_update": "k_rank_update (group labels; random 4-byte scatter)",
             "kasai": "k_kasai (LCP; random gathers)",
             "keyruns": "k_keys_runs (doubling keys sorted group by group in LDS)",
             "keybuild": "k_keys_dbl (doubling keys in text order)"}
    dom = max((k for k in keys if k in names), key=lambda k: kern[k]["ms"])
    L, ms, by = pkg.sa_timing_get(dom)
    achieved = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    traffic = None
    # counter-derived HBM bytes per launch (<kernel key>_traffic.json), valid only for the
    # source files the counters were taken on
    sources = {"radix_pass": ("radix.hip", "device.hpp"),
               "rank_update": ("sa_build.hip", "device.hpp", "internal.hpp")}
    tpath = os.path.join(args.traffic_dir, f"{dom}_traffic.json")
    if dom in sources and os.path.exists(tpath):
        import hashlib
        csrc = os.path.join(ROOT, "paper_1404_3456_amd", "csrc")
        h = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                    for f in sources[dom])).hexdigest()
        try:
            tr = json.load(open(tpath))
            if tr.get("source_sha256") == h and tuning is None and args.sa_algo == "doubling":
                traffic = tr.get("bytes_per_launch")
        except Exception:
            traffic = None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": names[dom],
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
        "sa_algorithm": args.sa_algo,
        ("sa_levels" if args.sa_algo == "dc3" else "sa_rounds"): rounds,
        "kernels": kern,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
