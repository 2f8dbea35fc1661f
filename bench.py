#!/usr/bin/env python3
"""Benchmark: one step = the whole hot path on one large job -- validate/pack, suffix array by
prefix doubling over LSD radix sorts, Kasai LCP, and suffix-prefix overlaps by LCP-interval
walks -- over the plain large workload (5 Mbp genome, 100,000 reads of 500 bp, 0.5 %
substitutions, N = 50.1 M suffixes, overlaps >= 40), input resident in HBM.

Prints one JSON line.  `value` is suffixes per second of the whole step (Msuffixes/s), timed
with no per-launch instrumentation.  Separate passes then measure:
  * the suffix-array build alone (`sa_build`: its time, and its bytes by the survey's per-unit
    figures and by the implementation's own model, against the HBM peak);
  * every kernel's launches, durations and units of work, with HIP events recorded on the
    launch stream; `roofline` reports the kernel with the most time per step;
  * `served`: the continuous-batching job server against the plain per-job path on a Poisson
    stream of assembly jobs (completed and offered jobs/s, p50/p99 latency);
  * `cpu_baseline`: the CPU oracle on bounded samples of the same recipe, all host threads and
    one thread, SA, LCP and overlaps timed separately.
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
    ap.add_argument("--no-serving", action="store_true",
                    help="plain workload: skip the served-jobs leg")
    ap.add_argument("--cpu-sample-scale", type=float, default=0.5,
                    help="all-core oracle sample, as a fraction of the workload")
    ap.add_argument("--cpu-serial-scale", type=float, default=0.2,
                    help="single-thread oracle sample, as a fraction of the workload")
    ap.add_argument("--kernel-steps", type=int, default=5,
                    help="steps of each instrumented pass (per-kernel times)")
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
    ap.add_argument("--pool", type=int, default=256, help="serving: distinct jobs generated")
    ap.add_argument("--jobs", type=int, default=2000,
                    help="serving: jobs per arrival-rate run (at least; rates above "
                         "jobs/6 per second run 6 s of arrivals)")
    ap.add_argument("--keep-up", type=float, default=0.98,
                    help="serving: a rate counts only if completed >= this x offered")
    ap.add_argument("--workers", type=int, default=8, help="serving: server worker streams")
    ap.add_argument("--max-jobs", type=int, default=64, help="serving: jobs per batch at most")
    ap.add_argument("--p99-bound-ms", type=float, default=500.0, help="serving: p99 bound")
    ap.add_argument("--patterns", type=int, default=1_000_000, help="lookup: patterns per step")
    ap.add_argument("--pattern-len", type=int, default=40, help="lookup: pattern length")
    ap.add_argument("--traffic-dir", default=os.path.join(ROOT, "profiles"),
                    help="folder of <kernel>_traffic.json files: HBM bytes per launch from rocprofv3 counters")
    return ap.parse_args()


def _host_cpu():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def _oracle_run(r, threads):
    import oracle
    t0 = time.perf_counter()
    sa = oracle.suffix_array(r.text, threads)
    t1 = time.perf_counter()
    lcp = oracle.lcp_array(r.text, sa, threads)
    t2 = time.perf_counter()
    ovl = oracle.overlaps(r.text, r.min_len, threads)
    t3 = time.perf_counter()
    return {"threads": threads, "n": r.n, "sample": r.name, "sa_s": round(t1 - t0, 3),
            "lcp_s": round(t2 - t1, 3), "overlaps_s": round(t3 - t2, 3),
            "overlap_rows": int(ovl.shape[0]),
            "sa_Msuffixes_per_s": round(r.n / (t1 - t0) / 1e6, 3),
            "Msuffixes_per_s": round(r.n / (t3 - t0) / 1e6, 3)}


def cpu_baseline(scale, serial_scale):
    """The oracle as it stands on the host: all threads on one sample, one thread (the paper's
    serial CPU comparison point) on a smaller one; SA, LCP and overlaps timed separately."""
    from paper_1404_3456_amd import synth
    model, nproc = _host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", nproc))
    threads = max(1, min(threads, nproc))
    allc = _oracle_run(synth.large_plain(scale=scale), threads)
    log(f"cpu baseline, {threads} threads: {allc}")
    serial = _oracle_run(synth.large_plain(scale=serial_scale), 1)
    log(f"cpu baseline, 1 thread: {serial}")
    return {
        "value": allc["Msuffixes_per_s"],
        "unit": "Msuffixes/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"plain-large-5M recipe at scale {scale:g} (N={allc['n']}, all {threads} "
                   f"threads) and at scale {serial_scale:g} (N={serial['n']}, one thread); "
                   f"SA + LCP + overlaps, each timed"),
        "host": {"cpu_model": model, "nproc": nproc},
        "modes": {"all_cores": allc, "single_thread": serial},
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
            text, off, candidates=[(9, 1024, 16), (8, 1024, 16), (9, 512, 16), (11, 512, 16)],
            seg_packs=(0, 1 << 28), reps=1, use_cache=False, log=log)
        log(f"autotuned: {tuning}")

    plain_tuning = None
    if tuning is not None and (tuning.digit_bits or tuning.block_threads or tuning.items_per_thread):
        plain_tuning = pkg.Tuning(tuning.digit_bits, tuning.block_threads, tuning.items_per_thread, 0)

    def batched():
        # the batched build computes the LCP array itself (its scan keeps to each set's block)
        sa, isa, lcp = pkg.sa_build_batched(text, off, tuning=tuning, use_graph=args.graph,
                                            lcp=True)
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
    pkg.sa_timing_reset()
    pkg.sa_timing_enable(True)
    batched()
    torch.cuda.synchronize()
    pkg.sa_timing_enable(False)
    kern = kernel_table(pkg, KEYS + ("big_place",), 1)
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
        "kernels": kern,
        "autotune": tune_report,
    }
    print(json.dumps(out), flush=True)


def _serving_text(job):
    from paper_1404_3456_amd import synth
    index, j, g = job
    return synth.serving_job(index, j, g).text


def serving_pool(n_pool):
    """The first n_pool jobs of the serving stream (genome log-uniform 1 kbp-5 Mbp, reads
    150-800 bp, 8x, 0.5 % substitutions), generated in parallel processes.  Call before the
    GPU is touched: the workers are fresh interpreters."""
    import concurrent.futures as cf
    import multiprocessing as mp
    from paper_1404_3456_amd import synth
    t0 = time.perf_counter()
    _, sizes = synth.serving_plan(n_jobs=n_pool, rate_per_s=1.0)
    jobs = [(3, j, g) for j, g in enumerate(sizes)]
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        texts = list(ex.map(_serving_text, jobs, chunksize=4))
    log(f"serving pool: {n_pool} jobs, {sum(t.size for t in texts)/1e6:.1f} M chars, "
        f"generated in {time.perf_counter()-t0:.1f} s on {workers} processes")
    return texts


def serving_measure(args, pkg, np, texts):
    """Open-loop Poisson arrivals of jobs drawn from `texts`, served by the continuous-batching
    server and by the plain path (one job at a time, single-text entry points), both under a
    64 GiB arena.  Latency = completion minus scheduled arrival.  A rate counts only when the
    server kept up with it: completed jobs/s >= keep_up x the offered (realised arrival) rate,
    and p99 within the bound."""
    import threading
    pool_n = len(texts)
    arena = 64 << 30

    def run(mode, rate, n_jobs, workers):
        # the same job sequence for every run; only the arrival times depend on the rate
        order = np.random.default_rng(1404).integers(0, pool_n, size=n_jobs)
        rng = np.random.default_rng(1404 + int(rate * 1000))
        gaps = rng.exponential(1.0 / rate, size=n_jobs) if rate > 0 else np.zeros(n_jobs)
        arr = np.cumsum(gaps) - gaps[0]
        lat = np.zeros(n_jobs)
        pending = {}
        lock = threading.Lock()
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

            th = threading.Thread(target=submitter)
            th.start()
            finished = 0
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
                if not items:
                    time.sleep(0.0002)
            th.join()
            stats = srv.asm_server_stats()
        span = float(np.max(arr + lat))  # first arrival to last completion
        out = {"mode": "plain" if mode == 1 else "served", "rate": round(rate, 2), "jobs": n_jobs,
               "completed_jobs_per_s": round(n_jobs / span, 2),
               "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
               "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
               "batches": stats["batches"],
               "max_concurrent_batches": stats["max_concurrent_batches"]}
        if rate > 0:
            out["offered_jobs_per_s"] = round((n_jobs - 1) / float(arr[-1]), 2)
            out["kept_up"] = bool(out["completed_jobs_per_s"]
                                  >= args.keep_up * out["offered_jobs_per_s"])
        return out

    def jobs_at(rate):
        return max(args.jobs, int(6 * rate))

    sat_p = run(1, 0.0, args.jobs, 1)
    mu_p = sat_p["completed_jobs_per_s"]
    log(f"plain saturated: {sat_p}")
    plain_pt = run(1, 0.8 * mu_p, max(1000, args.jobs // 2), 1)
    log(f"plain at 0.8x capacity: {plain_pt}")
    sat_s = run(0, 0.0, args.jobs, args.workers)
    log(f"served saturated: {sat_s}")
    bound_ms = args.p99_bound_ms
    points = []

    def point(k):
        """Served run at k x the plain capacity; True when it kept up within the p99 bound."""
        rate = k * mu_p
        if rate > 1.1 * sat_s["completed_jobs_per_s"]:
            return False
        pt = run(0, rate, jobs_at(rate), args.workers)
        pt["rate_x_plain"] = round(k, 4)
        points.append(pt)
        log(f"served {k:.3f}x: {pt}")
        return pt["kept_up"] and pt["p99_ms"] <= bound_ms

    # whole multiples of the plain capacity until one is not kept up, then three halvings of
    # the interval between the last rate kept up and the first one that was not
    lo = hi = None
    for k in (1.0, 2.0, 3.0, 4.0, 5.0, 6.0):
        if point(k):
            lo = k
        else:
            hi = k
            break
    if lo is not None and hi is not None:
        for _ in range(3):
            mid = 0.5 * (lo + hi)
            if point(mid):
                lo = mid
            else:
                hi = mid
    ok = [p for p in points if p["kept_up"] and p["p99_ms"] <= bound_ms]
    best = max(ok, key=lambda p: p["completed_jobs_per_s"]) if ok else None
    return {
        "jobs_per_s": best["completed_jobs_per_s"] if best else None,
        "offered_jobs_per_s": best["offered_jobs_per_s"] if best else None,
        "p50_ms": best["p50_ms"] if best else None,
        "p99_ms": best["p99_ms"] if best else None,
        "p99_bound_ms": bound_ms,
        "keep_up_rule": f"completed >= {args.keep_up} x offered",
        "plain_capacity_jobs_per_s": mu_p,
        "plain_at_0.8x": {k: plain_pt[k] for k in ("offered_jobs_per_s", "completed_jobs_per_s",
                                                   "p50_ms", "p99_ms", "kept_up")},
        "speedup_vs_plain": round(best["completed_jobs_per_s"] / mu_p, 3) if best else None,
        "served_saturated_jobs_per_s": sat_s["completed_jobs_per_s"],
        "saturated_speedup": round(sat_s["completed_jobs_per_s"] / mu_p, 3),
        "workload": "serving: Poisson jobs, genome log-uniform 1 kbp-5 Mbp, reads 150-800 bp, "
                    "8x, 0.5% subs, overlaps >= 40, 64 GiB arena",
        "pool": pool_n, "jobs_per_run_min": args.jobs, "workers": args.workers,
        "max_jobs_per_batch": args.max_jobs,
        "points": points,
    }


def bench_serving(args, pkg, torch, np, texts):
    """The served-jobs measurement as its own JSON line (see serving_measure)."""
    sv = serving_measure(args, pkg, np, texts)
    out = {
        "metric": "served jobs/s at p99 <= bound (kept up) vs plain per-job path",
        "value": sv["jobs_per_s"], "unit": "jobs/s",
        "n_gpus": 1, "steps": args.jobs, "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": sv["workload"], "pool": sv["pool"],
                   "jobs_per_run_min": args.jobs, "workers": args.workers,
                   "max_jobs_per_batch": args.max_jobs, "p99_bound_ms": args.p99_bound_ms},
        "served": sv,
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


# Bytes per unit of work by the survey's design estimate for each kernel (units as
# sa_timing_items counts them): the figures `roofline` and `sa_build` bill against the HBM peak.
# The library's own figures (what each kernel moves in this implementation) come beside them.
SURVEY_BYTES = {
    "pack": 1.375,        # read the byte, write 2 code bits and the separator bit
    "key0": 8.25,         # write an 8-byte first-round key from the 2-bit codes
    "radix_pass": 24.0,   # read and write an 8-byte key and a 4-byte value
    "keybuild": 20.0,     # doubling keys, per large-group item (read rank[p+h]; write key, value)
    "keyruns": 20.0,      # the same keys, built and ordered run by run
    "rank_update": 16.0,  # read key 8 + SA 4, write the rank 4, per active suffix
    "kasai": 12.0,        # isa 4 + the gathered sa 4 + the lcp write 4, per suffix
    "lcp_gather": 0.0,    # second half of the position-ordered LCP form (inside Kasai's 12)
}
KERNEL_NAMES = {
    "radix_pass": "k_onesweep (one LSD radix pass)",
    "rank_update": "k_rank_update (group labels; random 4-byte scatter)",
    "kasai": "k_kasai (LCP; random gathers)",
    "keyruns": "k_keys_runs (doubling keys sorted group by group in LDS)",
    "keybuild": "k_big_extract (doubling keys of the large groups' items)",
    "key0": "k_key0 (first-round keys + digit histograms)",
    "overlap_walk": "k_ovl_walk (LCP-interval walks)",
}
KEYS = ("pack", "key0", "radix_pass", "keybuild", "keyruns", "rank_update", "kasai",
        "lcp_gather", "overlap_walk")
BUILD_KEYS = ("pack", "key0", "radix_pass", "keybuild", "keyruns", "rank_update")


def kernel_table(pkg, keys, steps):
    out = {}
    for key in keys:
        L, ms, by = pkg.sa_timing_get(key)
        if not L:
            continue
        items = pkg.sa_timing_items(key)
        e = {"launches_per_step": round(L / steps, 2), "ms_per_step": round(ms / steps, 4),
             "avg_us": round(ms * 1000.0 / L, 3), "units_per_step": round(items / steps),
             "impl_bytes_per_step": round(by / steps), "impl_GBs": round(by / (ms * 1e-3) / 1e9, 1)}
        if key in SURVEY_BYTES:
            b8 = items * SURVEY_BYTES[key]
            e["survey_bytes_per_unit"] = SURVEY_BYTES[key]
            e["survey_bytes_per_step"] = round(b8 / steps)
            e["survey_GBs"] = round(b8 / (ms * 1e-3) / 1e9, 1)
        out[key] = e
    return out


def traffic_for(args, key, tuning):
    """Counter-measured HBM bytes per launch (<kernel key>_traffic.json under profiles/), valid
    only for the sources the counters were taken on and the default tuning."""
    import hashlib
    sources = {"radix_pass": ("radix.hip", "device.hpp"),
               "sa_build": ("sa_build.hip", "radix.hip", "pack.hip", "device.hpp", "internal.hpp"),
               "rank_update": ("sa_build.hip", "device.hpp", "internal.hpp"),
               "kasai": ("lcp.hip", "text.hpp", "device.hpp", "internal.hpp"),
               "keyruns": ("sa_build.hip", "device.hpp", "internal.hpp")}
    tpath = os.path.join(args.traffic_dir, f"{key}_traffic.json")
    if key not in sources or not os.path.exists(tpath) or tuning is not None:
        return None
    csrc = os.path.join(ROOT, "paper_1404_3456_amd", "csrc")
    h = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                for f in sources[key])).hexdigest()
    try:
        tr = json.load(open(tpath))
    except (OSError, ValueError):
        return None
    if tr.get("source_sha256") != h or args.sa_algo != "doubling":
        return None
    return tr.get("bytes_per_launch")


def copy_ceiling(pkg, torch, dev, reps=10):
    """The practical bandwidth ceiling: a 1 GiB device-to-device copy (1 GiB read + 1 GiB
    written per copy), timed with events on the stream the copies run on, by the runtime's own
    copy (torch `copy_`, hipMemcpyAsync device to device) and by the library's plain
    grid-stride copy kernel (the one the traffic counters are scaled by)."""
    words = 256 << 20
    src = torch.ones(words, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    moved = 2 * 4 * words
    out = {"bytes_per_copy": moved}
    for name, fn in (("runtime_copy", lambda: dst.copy_(src)),
                     ("k_copy_u32", lambda: pkg.sa_copy_u32(dst, src))):
        for _ in range(3):
            fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3 / reps
        out[name + "_GBs"] = round(moved / sec / 1e9, 1)
    out["GBs"] = max(out["runtime_copy_GBs"], out["k_copy_u32_GBs"])
    out["frac_of_peak"] = round(out["GBs"] / HBM_PEAK_GBS, 4)
    del src, dst
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                          "(the design for more GPUs is described, not run)"}))
        sys.exit(2)
    import numpy as np
    from paper_1404_3456_amd import synth

    # the serving pool is generated in worker processes before this process touches the GPU
    serving_texts = None
    if args.workload == "serving" or (args.workload == "plain-large-5M" and not args.no_serving):
        serving_texts = serving_pool(args.pool)

    import torch
    import paper_1404_3456_amd as pkg

    pkg.load()
    if args.workload == "batched-256":
        return bench_batched(args, pkg, torch, np)
    if args.workload == "serving":
        return bench_serving(args, pkg, torch, np, serving_texts)
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

    def build_sa():
        if args.sa_algo == "dc3":
            return pkg.sa_build_dc3(text, tuning=tuning, return_levels=True)
        return pkg.sa_build(text, tuning=tuning, return_rounds=True)

    def step():
        sa, isa, rounds = build_sa()
        lcp = pkg.sa_lcp(text, sa, isa)
        ovl = pkg.sa_overlaps(text, sa, isa, lcp, r.min_len)
        return sa, isa, lcp, ovl, rounds

    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            pkg.sa_copy_u32(dst, src)
        torch.cuda.synchronize()
        log("calibration copy: 3 x 256 MiB read + 256 MiB written")
    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i} done")

    # 1. the timed steps: no instrumentation inside
    pkg.sa_timing_enable(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        sa, isa, lcp, ovl, rounds = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step")

    # 2. the suffix-array build alone, uninstrumented (each build synchronised)
    ks = max(1, args.kernel_steps)
    build_ms = []
    for _ in range(ks):
        torch.cuda.synchronize()
        a = time.perf_counter()
        build_sa()
        torch.cuda.synchronize()
        build_ms.append((time.perf_counter() - a) * 1e3)
    sa_build_ms = float(np.median(build_ms))

    # 3. the build alone with per-launch events: its kernels' bytes
    pkg.sa_timing_reset()
    pkg.sa_timing_enable(True)
    for _ in range(ks):
        build_sa()
    torch.cuda.synchronize()
    pkg.sa_timing_enable(False)
    build_kern = kernel_table(pkg, BUILD_KEYS, ks)
    b8 = sum(e.get("survey_bytes_per_step", 0) for e in build_kern.values())
    bimpl = sum(e["impl_bytes_per_step"] for e in build_kern.values())
    # the build's counted traffic (all its kernels, one build) where it was taken on these sources
    btr = traffic_for(args, "sa_build", tuning)
    sa_build = {
        "ms": round(sa_build_ms, 3),
        "traffic": btr,
        "traffic_GBs": round(btr / (sa_build_ms * 1e-3) / 1e9, 1) if btr else None,
        "traffic_frac": round(btr / (sa_build_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if btr else None,
        "Msuffixes_per_s": round(n / (sa_build_ms * 1e-3) / 1e6, 3),
        "survey_bytes": b8,
        "achieved_GBs": round(b8 / (sa_build_ms * 1e-3) / 1e9, 1),
        "frac": round(b8 / (sa_build_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "impl_bytes": bimpl,
        "impl_GBs": round(bimpl / (sa_build_ms * 1e-3) / 1e9, 1),
        "impl_frac": round(bimpl / (sa_build_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "peak_GBs": HBM_PEAK_GBS,
        "kernels": build_kern,
        "note": "bytes = units of work x bytes per unit, by the survey's per-kernel figures "
                "(survey_*) and by the implementation's own model (impl_*), over the build's "
                "time with no instrumentation; traffic = FETCH_SIZE + WRITE_SIZE of every kernel "
                "of one build, counted at the L2 boundary (profiles/sa_build_traffic.json)",
    }
    log(f"SA build alone: {sa_build_ms:.3f} ms, {sa_build['frac']:.3f} of peak (survey bytes)")

    # 4. whole steps with per-launch events: the dominant kernel
    pkg.sa_timing_reset()
    pkg.sa_timing_enable(True)
    for _ in range(ks):
        step()
    torch.cuda.synchronize()
    pkg.sa_timing_enable(False)
    kern = kernel_table(pkg, KEYS + (("dc3_keys", "dc3_names", "dc3_lift", "dc3_recs",
                                       "dc3_merge") if args.sa_algo == "dc3" else ()), ks)
    dom = max((k for k in kern if k in KERNEL_NAMES), key=lambda k: kern[k]["ms_per_step"])
    d = kern[dom]
    L, ms, by = pkg.sa_timing_get(dom)
    items = pkg.sa_timing_items(dom)
    avg_s = ms * 1e-3 / L
    per_unit = SURVEY_BYTES.get(dom)
    alg = items / L * per_unit if per_unit is not None else by / L
    traffic = traffic_for(args, dom, tuning)
    roofline = {"bound": "hbm", "achieved": round(alg / avg_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(alg / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                # the counted bytes over the same launch time: how busy the memory side is
                "traffic_GBs": round(traffic / avg_s / 1e9, 1) if traffic else None,
                "traffic_frac": round(traffic / avg_s / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
                "kernel": KERNEL_NAMES[dom],
                "units_per_launch": round(items / L),
                "bytes_per_unit": per_unit,
                "alg_bytes_per_launch": round(alg),
                "avg_launch_us": round(avg_s * 1e6, 3),
                "impl_bytes_per_launch": round(by / L),
                "impl_achieved": round(by / L / avg_s / 1e9, 1),
                "impl_frac": round(by / L / avg_s / 1e9 / HBM_PEAK_GBS, 4)}
    log(f"dominant kernel {dom}: {d}")

    copy = copy_ceiling(pkg, torch, dev)
    log(f"copy ceiling: {copy}")
    if sa_build.get("traffic_GBs"):
        sa_build["traffic_vs_copy"] = round(sa_build["traffic_GBs"] / copy["GBs"], 4)
    sa_build["survey_vs_copy"] = round(sa_build["achieved_GBs"] / copy["GBs"], 4)

    served = None
    if serving_texts is not None:
        log("served-jobs leg ...")
        served = serving_measure(args, pkg, np, serving_texts)
        log(f"served: {served['jobs_per_s']} jobs/s vs plain {served['plain_capacity_jobs_per_s']}")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(args.cpu_sample_scale, args.cpu_serial_scale)
        log(f"cpu baseline: {cpu['value']} Msuffixes/s on {cpu['cores']} threads")

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
        "sa_algorithm": args.sa_algo,
        ("sa_levels" if args.sa_algo == "dc3" else "sa_rounds"): rounds,
        "sa_build": sa_build,
        "kernels": kern,
        "roofline": roofline,
        "copy_ceiling": copy,
        "served": served,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
