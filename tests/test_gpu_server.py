"""GPU tests of the job server: results identical alone and in a mix, bad jobs rejected with the
server still running, an injected allocation failure fails only its batch."""
import time

import numpy as np
import pytest

import oracle
from paper_1404_3456_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pkg():
    import paper_1404_3456_amd as p
    p.load()
    return p


def wait(srv, jid, timeout=120.0):
    t0 = time.time()
    while True:
        r = srv.asm_poll(jid)
        if r is not None:
            return r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"job {jid}")
        time.sleep(0.001)


def host(r):
    return (r["sa"].cpu().numpy(), r["isa"].cpu().numpy(), r["lcp"].cpu().numpy(),
            r["ovl"].cpu().numpy())


def jobs_pool(k, seed=3):
    out = []
    rng = np.random.default_rng(seed)
    for j in range(k):
        g = int(rng.integers(500, 30_000))
        out.append(synth.genome_reads(seed * 100 + j, g, int(rng.integers(5, 200)),
                                      int(rng.integers(30, min(300, g))), err=0.005))
    return out


@pytest.mark.parametrize("mode,workers", [(0, 1), (0, 3), (1, 1)])
def test_server_results_match_oracle(pkg, mode, workers):
    texts = jobs_pool(12)
    with pkg.AsmServer(1 << 30, max_jobs_per_batch=8, workers=workers, mode=mode) as srv:
        ids = [srv.asm_submit(t, 20) for t in texts]
        for jid, t in zip(ids, texts):
            r = wait(srv, jid)
            assert r["status"] == 0
            sa, isa, lcp, ovl = host(r)
            want = oracle.suffix_array(t)
            assert np.array_equal(sa, want)
            assert np.array_equal(isa[sa], np.arange(t.size))
            assert np.array_equal(lcp, oracle.lcp_array(t, want))
            assert np.array_equal(ovl, oracle.overlaps(t, 20))
            assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
            srv.asm_release(jid)
        st = srv.asm_server_stats()
        assert st["jobs_done"] == len(texts) and st["arena_used"] == 0


def test_same_result_alone_and_in_mix(pkg):
    texts = jobs_pool(20, seed=8)
    probe = texts[7]
    with pkg.AsmServer(1 << 30, max_jobs_per_batch=32, workers=2) as srv:
        alone = srv.asm_submit(probe, 25)
        ra = host(wait(srv, alone))
        ids = [srv.asm_submit(t, 25) for t in texts]  # probe again, now inside a mix
        rm = host(wait(srv, ids[7]))
        for a, b in zip(ra, rm):
            assert np.array_equal(a, b)
        for jid in ids:
            wait(srv, jid)
        assert srv.asm_server_stats()["batches"] < 1 + len(texts)  # jobs were batched


def test_bad_jobs_rejected_server_keeps_running(pkg):
    with pkg.AsmServer(1 << 28, workers=1) as srv:
        with pytest.raises(pkg.SaasmError) as e:
            srv.asm_submit(np.frombuffer(b"ACGN$", dtype=np.uint8), 3)
        assert e.value.code == pkg.SA_ERR_ALPHABET
        with pytest.raises(pkg.SaasmError):
            srv.asm_submit(np.frombuffer(b"ACGT", dtype=np.uint8), 3)
        big = np.full(50_000_000, ord("A"), dtype=np.uint8)
        big[-1] = ord("$")
        with pytest.raises(pkg.SaasmError) as e:
            srv.asm_submit(big, 3)  # over the 256 MiB budget
        assert e.value.code == pkg.SA_ERR_NOMEM
        t = jobs_pool(1)[0]
        r = wait(srv, srv.asm_submit(t, 20))
        assert r["status"] == 0
        assert np.array_equal(host(r)[0], oracle.suffix_array(t))


def test_injected_alloc_failure_fails_one_batch_only(pkg):
    texts = jobs_pool(6, seed=11)
    with pkg.AsmServer(1 << 30, max_jobs_per_batch=1, workers=1) as srv:
        srv.fail_alloc_after(1)  # the next batch's first allocation fails
        first = srv.asm_submit(texts[0], 20)
        r0 = wait(srv, first)
        assert r0["status"] == pkg.SA_ERR_NOMEM
        ids = [srv.asm_submit(t, 20) for t in texts[1:]]
        for jid, t in zip(ids, texts[1:]):
            r = wait(srv, jid)
            assert r["status"] == 0
            assert np.array_equal(host(r)[0], oracle.suffix_array(t))
            srv.asm_release(jid)
        srv.asm_release(first)
        assert srv.asm_server_stats()["arena_used"] == 0


def test_borrowed_texts_and_deferred_rejection(pkg):
    texts = jobs_pool(6, seed=21)
    bad = np.frombuffer(b"ACGTN$ACG$", dtype=np.uint8).copy()
    with pkg.AsmServer(1 << 30, max_jobs_per_batch=8, workers=2) as srv:
        ids = [srv.asm_submit(t, 20, borrow=True) for t in texts[:3]]
        bad_id = srv.asm_submit(bad, 3, borrow=True)  # accepted, fails when run
        ids += [srv.asm_submit(t, 20, borrow=True) for t in texts[3:]]
        assert wait(srv, bad_id)["status"] == pkg.SA_ERR_ALPHABET
        for jid, t in zip(ids, texts):
            r = wait(srv, jid)
            assert r["status"] == 0
            sa, isa, lcp, ovl = host(r)
            assert np.array_equal(sa, oracle.suffix_array(t))
            assert np.array_equal(ovl, oracle.overlaps(t, 20))
            srv.asm_release(jid)
        srv.asm_release(bad_id)
        assert srv.asm_server_stats()["arena_used"] == 0


def test_full_serving_jobs(pkg):
    """The serving workload's first 64 jobs (genome 1 kbp-5 Mbp log-uniform, reads 150-800 bp,
    8x, 0.5 % substitutions) submitted at once to a server with the benchmark's 64 GiB arena,
    4 workers and batches of up to 64 jobs: every job against the oracle -- SA and LCP equal to
    the oracle's arrays up to 2 M characters and, above, a permutation whose every adjacent pair
    ascends with the direct LCP (the same definition, checked pair by pair) -- and the overlaps
    (>= 40) exactly."""
    _, jobs = synth.serving_jobs(n_jobs=64, rate_per_s=1.0)
    print(f"full-size serving: {len(jobs)} jobs, {sum(j.n for j in jobs)} characters", flush=True)
    with pkg.AsmServer(64 << 30, max_jobs_per_batch=64, workers=4, mode=0) as srv:
        ids = [srv.asm_submit(j.text, 40) for j in jobs]
        for jid, job in zip(ids, jobs):
            r = wait(srv, jid, timeout=300.0)
            assert r["status"] == 0, job.name
            sa, isa, lcp, ovl = host(r)
            t = job.text
            assert np.array_equal(isa[sa], np.arange(t.size)), job.name
            if t.size <= 2_000_000:
                want = oracle.suffix_array(t)
                assert np.array_equal(sa, want), job.name
                assert np.array_equal(lcp, oracle.lcp_array(t, want)), job.name
            else:
                # a permutation whose adjacent suffixes all ascend is the suffix array
                assert np.all(np.bincount(sa, minlength=t.size) == 1), job.name
                bad, first = oracle.check_all(t, sa, lcp)
                assert bad == 0, (job.name, bad, first)
                assert lcp[0] == 0, job.name
            assert np.array_equal(ovl, oracle.overlaps(t, 40)), job.name
            srv.asm_release(jid)
        st = srv.asm_server_stats()
        assert st["jobs_done"] == len(jobs) and st["arena_used"] == 0


def test_failure_inside_a_running_batch(pkg):
    """An allocation that fails inside a batch already on the device (the overlap rows, the
    third allocation of a batch): that batch's jobs fail with SA_ERR_NOMEM after its queued
    kernels have finished, its memory comes back, and later jobs on the other workers are
    exact."""
    texts = jobs_pool(8, seed=13)
    with pkg.AsmServer(1 << 30, max_jobs_per_batch=4, workers=2) as srv:
        srv.fail_alloc_after(3)
        first = srv.asm_submit(texts[0], 20)
        assert wait(srv, first)["status"] == pkg.SA_ERR_NOMEM
        srv.asm_release(first)
        assert srv.asm_server_stats()["arena_used"] == 0
        ids = [srv.asm_submit(t, 20) for t in texts[1:]]
        for jid, t in zip(ids, texts[1:]):
            r = wait(srv, jid)
            assert r["status"] == 0
            sa, isa, lcp, ovl = host(r)
            want = oracle.suffix_array(t)
            assert np.array_equal(sa, want)
            assert np.array_equal(lcp, oracle.lcp_array(t, want))
            assert np.array_equal(ovl, oracle.overlaps(t, 20))
            srv.asm_release(jid)
        st = srv.asm_server_stats()
        assert st["arena_used"] == 0 and st["jobs_done"] == len(texts)


def test_batching_resumes_after_a_job_too_large_to_share(pkg):
    """The arena holds the large job alone but not with any other: its batch shrinks until it
    runs alone, then the small jobs behind it are batched again at the full batch size.  The
    client copies every result out and releases it at once; the oracle checks run after all
    jobs are back."""
    big = synth.genome_reads(901, 300_000, 6000, 500, err=0.005)     # ~3 M characters
    smalls = [synth.genome_reads(910 + k, 20_000, 400, 250, err=0.005) for k in range(40)]
    n, ns = big.size, smalls[0].size
    # what the server holds for one job: text, SA, ISA, LCP (13 bytes per character) and the
    # batch scratch (the batched build's workspace, which includes the LCP's), plus the
    # overlap rows; 3 MiB over that is less than one small job adds (~5 MB)
    keep = 13 * n + 4 * 256
    scratch = max(pkg.sa_build_batched_ws_bytes(n, 1), pkg.sa_lcp_ws_bytes(n)) + 4096
    arena = keep + scratch + (n // 32 + 4096) * 12 + (3 << 20)
    both = 13 * (n + ns) + 2048 + pkg.sa_build_batched_ws_bytes(n + ns, 2) + 4096
    assert both > arena
    # 16 small jobs fit beside the large job's results and one earlier batch's results
    b16 = 16 * (13 * ns + 1024) + pkg.sa_build_batched_ws_bytes(16 * ns, 16) + 4096
    assert keep + 16 * (13 * ns + 1024) + b16 < arena
    got, res = [], []
    with pkg.AsmServer(arena, max_jobs_per_batch=16, workers=1) as srv:
        ids = [srv.asm_submit(big, 40)] + [srv.asm_submit(t, 40) for t in smalls]
        for jid in ids:
            r = wait(srv, jid, timeout=300.0)
            assert r["status"] == 0
            got.append(host(r))
            res.append(r)
            srv.asm_release(jid)
        st = srv.asm_server_stats()
    assert st["jobs_done"] == 41 and st["arena_used"] == 0
    # the large job ran alone: every small job was admitted after it finished
    assert min(r["t_admit"] for r in res[1:]) >= res[0]["t_done"]
    # then the small ones shared batches again (16 at a time: 3 batches; one job per batch
    # would make 41)
    assert st["batches"] <= 1 + 40 // 8, st
    for (sa, isa, lcp, ovl), t in zip(got, [big] + smalls):
        want = oracle.suffix_array(t)
        assert np.array_equal(sa, want)
        assert np.array_equal(lcp, oracle.lcp_array(t, want))
        assert np.array_equal(ovl, oracle.overlaps(t, 40))


def test_batches_fill_to_the_batch_size(pkg):
    """A 20 M-character job keeps the one worker busy while 40 small jobs queue behind it; with
    batches of up to 64 jobs the small ones are admitted together, so the whole run takes at
    most two batches (a cap below the batch size, e.g. 16 jobs, would need three or more)."""
    huge = synth.genome_reads(931, 2_000_000, 40_000, 500, err=0.005)
    smalls = [synth.genome_reads(940 + k, 20_000, 200, 250, err=0.005) for k in range(40)]
    with pkg.AsmServer(4 << 30, max_jobs_per_batch=64, workers=1) as srv:
        ids = [srv.asm_submit(huge, 40, borrow=True)]
        ids += [srv.asm_submit(t, 40, borrow=True) for t in smalls]
        got = []
        for jid in ids:
            r = wait(srv, jid, timeout=300.0)
            assert r["status"] == 0
            got.append(host(r))
            srv.asm_release(jid)
        st = srv.asm_server_stats()
    assert st["jobs_done"] == 41 and st["arena_used"] == 0
    assert st["batches"] <= 2, st
    for (sa, isa, lcp, ovl), t in zip(got[1:], smalls):
        want = oracle.suffix_array(t)
        assert np.array_equal(sa, want)
        assert np.array_equal(lcp, oracle.lcp_array(t, want))
        assert np.array_equal(ovl, oracle.overlaps(t, 40))
    sa, isa, lcp, ovl = got[0]
    assert np.array_equal(isa[sa], np.arange(huge.size))
    bad, first = oracle.check_all(huge, sa, lcp)
    assert bad == 0, (bad, first)
    assert np.array_equal(ovl, oracle.overlaps(huge, 40))


def test_mixed_min_len_jobs(pkg):
    """Jobs with two minimum overlap lengths interleaved in the queue: a batch holds one length
    and passes over (at most 16) queued jobs of the other, which keep their place; every job's
    SA, LCP and overlaps (at its own length) equal the oracle's."""
    texts = jobs_pool(30, seed=41)
    lens = [20 if (k % 3) else 35 for k in range(len(texts))]
    with pkg.AsmServer(1 << 30, max_jobs_per_batch=64, workers=2) as srv:
        ids = [srv.asm_submit(t, L, borrow=True) for t, L in zip(texts, lens)]
        for jid, t, L in zip(ids, texts, lens):
            r = wait(srv, jid)
            assert r["status"] == 0
            sa, isa, lcp, ovl = host(r)
            want = oracle.suffix_array(t)
            assert np.array_equal(sa, want)
            assert np.array_equal(lcp, oracle.lcp_array(t, want))
            assert np.array_equal(ovl, oracle.overlaps(t, L)), (jid, L)
            srv.asm_release(jid)
        st = srv.asm_server_stats()
    assert st["jobs_done"] == len(texts) and st["arena_used"] == 0
