"""GPU parity: every result of the HIP library, called through the C ABI, against the CPU
oracle on the same seeded inputs.  Integer work throughout, so every comparison is exact."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1404_3456_amd import synth
from tests import checks

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    import paper_1404_3456_amd as pkg
    pkg.load()
    return pkg


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_sa(lib, text, tuning=None):
    sa, isa = lib.sa_build(dev(text), tuning=tuning)
    torch.cuda.synchronize()
    return sa.cpu().numpy(), isa.cpu().numpy()


def run_all(lib, text, min_len, tuning=None):
    t = dev(text)
    sa, isa = lib.sa_build(t, tuning=tuning)
    lcp = lib.sa_lcp(t, sa, isa)
    ovl = lib.sa_overlaps(t, sa, isa, lcp, min_len)
    torch.cuda.synchronize()
    return sa.cpu().numpy(), isa.cpu().numpy(), lcp.cpu().numpy(), ovl.cpu().numpy()


def assert_parity(lib, text, min_len=1, tuning=None, label=""):
    sa, isa, lcp, ovl = run_all(lib, text, min_len, tuning)
    want_sa = oracle.suffix_array(text)
    assert np.array_equal(sa, want_sa), f"SA mismatch {label}"
    assert np.array_equal(isa[sa], np.arange(text.size)), f"ISA mismatch {label}"
    want_lcp = oracle.lcp_array(text, want_sa)
    assert np.array_equal(lcp, want_lcp), f"LCP mismatch {label}"
    want_ovl = oracle.overlaps(text, min_len)
    assert np.array_equal(ovl.reshape(-1, 3), want_ovl), f"overlap mismatch {label}"


# ---- packing -------------------------------------------------------------------------------

def test_pack_layout(lib):
    text = synth.random_dna_reads(1, 300, 0, 70, allow_empty=True)
    packed, sepmask, read_end = lib.sa_pack(dev(text))
    packed = packed.cpu().numpy().view(np.uint32)
    sepmask = sepmask.cpu().numpy().view(np.uint32)
    n = text.size
    lut = np.zeros(256, dtype=np.uint32)
    lut[ord("C")], lut[ord("G")], lut[ord("T")] = 1, 2, 3
    codes = lut[text]
    pad = np.zeros(packed.size * 16, dtype=np.uint32)
    pad[:n] = codes
    want_p = (pad.reshape(-1, 16) << (30 - 2 * np.arange(16, dtype=np.uint32))).sum(1).astype(np.uint32)
    assert np.array_equal(packed, want_p)
    sep = np.zeros(sepmask.size * 32, dtype=np.uint64)
    sep[:n] = text == ord("$")
    want_s = (sep.reshape(-1, 32) << (31 - np.arange(32, dtype=np.uint64))).sum(1).astype(np.uint32)
    assert np.array_equal(sepmask, want_s)
    assert np.array_equal(read_end.cpu().numpy(), np.flatnonzero(text == ord("$")))


def test_pack_rejects_bad_text(lib):
    with pytest.raises(lib.SaasmError) as e:
        lib.sa_pack(dev(np.frombuffer(b"ACGN$", dtype=np.uint8).copy()))
    assert e.value.code == lib.SA_ERR_ALPHABET
    with pytest.raises(lib.SaasmError) as e:
        lib.sa_build(dev(np.frombuffer(b"ACGT$acgt$", dtype=np.uint8).copy()))
    assert e.value.code == lib.SA_ERR_ALPHABET
    with pytest.raises(lib.SaasmError) as e:
        lib.sa_build(dev(np.frombuffer(b"ACGT$AC", dtype=np.uint8).copy()))
    assert e.value.code == lib.SA_ERR_INVALID


# ---- radix sort: one pass is a stable counting sort; the whole sort is a stable sort ---------

@pytest.mark.parametrize("tuning", [None, {"digit_bits": 4}, {"digit_bits": 9}, {"digit_bits": 11},
                                    {"block_threads": 512, "items_per_thread": 16},
                                    {"block_threads": 512, "items_per_thread": 8},
                                    {"block_threads": 256, "items_per_thread": 8}])
@pytest.mark.parametrize("bits", [(0, 64), (0, 8), (3, 14), (32, 49), (60, 64)])
def test_sort_pairs_stable(lib, tuning, bits):
    rng = np.random.default_rng(abs(hash((str(tuning), bits))) % (1 << 31))
    n = 70_001
    keys = rng.integers(0, 1 << 63, size=n, dtype=np.int64)
    keys[::7] = keys[3]  # many equal fields
    vals = np.arange(n, dtype=np.int32)
    lo, hi = bits
    field = (keys.view(np.uint64) >> np.uint64(lo))
    if hi - lo < 64:
        field &= np.uint64((1 << (hi - lo)) - 1)
    order = np.argsort(field, kind="stable")
    k_t, v_t = dev(keys.copy()), dev(vals.copy())
    lib.sa_sort_pairs(k_t, v_t, lo, hi, tuning=tuning)
    assert np.array_equal(v_t.cpu().numpy(), vals[order])
    assert np.array_equal(k_t.cpu().numpy(), keys[order])


@pytest.mark.parametrize("n", [0, 1, 2, 255, 4096, 4097, 65536 * 3 + 17])
def test_sort_pairs_sizes(lib, n):
    rng = np.random.default_rng(n)
    keys = rng.integers(0, 1 << 40, size=n, dtype=np.int64)
    vals = rng.integers(0, 1 << 31, size=n, dtype=np.int32)
    order = np.argsort(keys, kind="stable")
    if n == 0:
        return
    k_t, v_t = dev(keys.copy()), dev(vals.copy())
    lib.sa_sort_pairs(k_t, v_t, 0, 40)
    assert np.array_equal(k_t.cpu().numpy(), keys[order])
    assert np.array_equal(v_t.cpu().numpy(), vals[order])


# ---- suffix array / LCP / overlaps ----------------------------------------------------------

def tiny_dna_texts(max_len=6):
    out = []
    for L in range(0, max_len):
        for body in itertools.product("ACGT$", repeat=L):
            s = "".join(body) + "$"
            out.append(np.frombuffer(s.encode(), dtype=np.uint8).copy())
    return out


def test_tiny_exhaustive(lib):
    texts = tiny_dna_texts(5)
    rng = np.random.default_rng(5)
    texts += [t for t in tiny_dna_texts(6) if rng.random() < 0.05]
    for t in texts:
        sa, isa, lcp, ovl = run_all(lib, t, 1)
        want = oracle.suffix_array(t)
        assert np.array_equal(sa, want), t.tobytes()
        assert np.array_equal(isa[sa], np.arange(t.size)), t.tobytes()
        assert np.array_equal(lcp, oracle.lcp_array(t, want)), t.tobytes()
        assert np.array_equal(ovl.reshape(-1, 3), oracle.overlaps_brute(t, 1)), t.tobytes()


EDGE = {
    "one_sep": b"$",
    "two_seps": b"$$",
    "one_base": b"A$",
    "empty_reads": b"$AC$$GT$$",
    "homopolymer_10k": b"A" * 10_000 + b"$",
    "two_identical": b"ACGTTGCAAC$ACGTTGCAAC$",
    "many_identical": b"GATTACA$" * 300,
    "period3_5k": b"ACG" * 1700 + b"$",
    "two_homopolymers": b"A" * 3000 + b"$" + b"A" * 2999 + b"$",
    "nested": b"ACGTACGTACGT$CGTACG$GTAC$T$",
}


@pytest.mark.parametrize("name", sorted(EDGE))
def test_edge_cases(lib, name):
    t = np.frombuffer(EDGE[name], dtype=np.uint8).copy()
    assert_parity(lib, t, min_len=1, label=name)
    assert_parity(lib, t, min_len=3, label=name)


@pytest.mark.parametrize("seed,m,lo,hi,alpha", [
    (11, 200, 0, 50, b"ACGT"),
    (12, 400, 0, 120, b"AC"),
    (13, 2000, 1, 30, b"A"),
    (14, 50, 500, 2000, b"ACGT"),
    (15, 3000, 0, 40, b"ACG"),
])
def test_ragged_random(lib, seed, m, lo, hi, alpha):
    t = synth.random_dna_reads(seed, m, lo, hi, alphabet=alpha, allow_empty=True)
    assert_parity(lib, t, min_len=4, label=f"seed{seed}")


def text_of_length(seed, n):
    """Overlapping reads of a random genome (8x), cut to exactly n characters ending in '$'."""
    t = synth.genome_reads(seed, max(200, n // 8), max(4, n // 60), 60, err=0.01)
    while t.size < n:
        t = np.concatenate([t, synth.genome_reads(seed + t.size, max(200, n // 8), max(4, n // 60), 60)])
    t = t[:n].copy()
    t[-1] = ord("$")
    return t


@pytest.mark.parametrize("n", [2047, 2048, 2049, 8191, 8192, 8193, 16383, 16384, 16385, 24577])
def test_lengths_at_tile_boundaries(lib, n):
    """Texts whose length sits on either side of the tile sizes of the run sort (2,048 items), the
    rank update (8,192) and the radix pass (16,384): round 0 has all n suffixes active, so its
    last tile is full, a single item, or one short."""
    t = text_of_length(n, n)
    assert t.size == n and t[-1] == ord("$")
    assert_parity(lib, t, min_len=10, label=f"n={n}")


@pytest.mark.parametrize("seed", range(4))
def test_overlapping_reads(lib, seed):
    t = synth.genome_reads(seed, 3000 + 1000 * seed, 300, 80 + 20 * seed, err=0.01 * (seed % 2),
                           alphabet_size=2 + seed % 3)
    assert_parity(lib, t, min_len=15, label=f"genome{seed}")


def test_small_plain_workload(lib):
    r = synth.small_plain()
    assert_parity(lib, r.text, min_len=r.min_len, label=r.name)
    # and the positional ground truth for error-free equal-length reads
    t = dev(r.text)
    sa, isa = lib.sa_build(t)
    lcp = lib.sa_lcp(t, sa, isa)
    ovl = lib.sa_overlaps(t, sa, isa, lcp, r.min_len).cpu().numpy()
    assert np.array_equal(ovl, checks.positional_overlaps(r.starts, 200, r.min_len))


TUNINGS = [{"digit_bits": d, "block_threads": b, "items_per_thread": i}
           for d in (4, 8, 9, 11) for b, i in ((256, 8), (256, 16), (512, 8), (512, 16), (1024, 16))
           if not (b == 1024 and d > 9)]


def test_tunings_identical(lib):
    """Every digit width and tile shape gives byte-identical results (also a race check)."""
    t = synth.genome_reads(99, 20_000, 600, 150, err=0.005)
    want = oracle.suffix_array(t)
    for tu in TUNINGS:
        sa, _ = run_sa(lib, t, tu)
        assert np.array_equal(sa, want), tu


def test_repeat_runs_identical(lib):
    t = synth.genome_reads(7, 50_000, 2000, 100, err=0.005)
    first = run_all(lib, t, 20)
    for _ in range(3):
        again = run_all(lib, t, 20)
        for a, b in zip(first, again):
            assert np.array_equal(a, b)


# ---- LCP through the position-ordered form (the one texts above 2^26 positions take) ---------

def test_lcp_position_ordered_form(lib):
    prev = lib.sa_lcp_plcp_min(0)
    try:
        for name in sorted(EDGE):
            assert_parity(lib, np.frombuffer(EDGE[name], dtype=np.uint8).copy(), min_len=3,
                          label=name)
        assert_parity(lib, synth.random_dna_reads(11, 200, 0, 50, allow_empty=True), 4)
        for seed in range(2):
            t = synth.genome_reads(seed, 3000 + 1000 * seed, 300, 80 + 20 * seed, err=0.01 * seed)
            assert_parity(lib, t, min_len=15, label=f"genome{seed}")
        for chunk in (1, 16):
            lib.sa_lcp_set_chunk(chunk)
            try:
                r = synth.small_plain()
                assert_parity(lib, r.text, min_len=r.min_len, label=f"chunk {chunk}")
            finally:
                lib.sa_lcp_set_chunk(4)
    finally:
        lib.sa_lcp_plcp_min(prev)


# ---- batched build: many independent texts in one set of launches ---------------------------

def _batched_case(seed, n_sets, g_lo=200, g_hi=4000):
    rng = np.random.default_rng(seed)
    texts = []
    for s in range(n_sets):
        g = int(rng.integers(g_lo, g_hi))
        m = int(rng.integers(1, 40))
        L = int(rng.integers(5, min(120, g)))
        texts.append(synth.genome_reads(seed * 1000 + s, g, m, L, err=0.01 * (s % 2),
                                        alphabet_size=2 + s % 3))
    off = np.concatenate([[0], np.cumsum([t.size for t in texts])]).astype(np.int64)
    return texts, off, np.concatenate(texts)


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("seed,n_sets", [(1, 1), (2, 7), (3, 64), (4, 300)])
def test_batched_parity(lib, seed, n_sets, use_graph):
    texts, off, cat = _batched_case(seed, n_sets)
    t = dev(cat)
    sa, isa = lib.sa_build_batched(t, off, use_graph=use_graph)
    lcp = lib.sa_lcp(t, sa, isa)
    ovl = lib.sa_overlaps(t, sa, isa, lcp, 4).cpu().numpy()
    sa, isa, lcp = sa.cpu().numpy(), isa.cpu().numpy(), lcp.cpu().numpy()
    assert np.array_equal(isa[sa], np.arange(cat.size))
    reads_before = 0
    rows = []
    for s, txt in enumerate(texts):
        lo, hi = off[s], off[s + 1]
        want_sa = oracle.suffix_array(txt)
        assert np.array_equal(sa[lo:hi] - lo, want_sa), f"set {s}"
        assert np.array_equal(lcp[lo:hi], oracle.lcp_array(txt, want_sa)), f"set {s} lcp"
        o = oracle.overlaps(txt, 4).astype(np.int64)
        o[:, :2] += reads_before
        rows.append(o)
        reads_before += int((txt == ord("$")).sum())
    want = np.concatenate(rows) if rows else np.zeros((0, 3))
    assert np.array_equal(ovl.astype(np.int64), want)


@pytest.mark.parametrize("seg_pack,use_graph", [(0, False), (0, True), (20_000, False)])
def test_batched_lcp_output(lib, seg_pack, use_graph):
    """The LCP computed inside sa_build_batched (one build, or several packed builds whose LCP
    lands at their offsets) equals sa_lcp over the concatenation and the oracle per set."""
    texts, off, cat = _batched_case(21, 40)
    t = dev(cat)
    tu = {"seg_pack": seg_pack} if seg_pack else None
    sa, isa, lcp = lib.sa_build_batched(t, off, tuning=tu, use_graph=use_graph, lcp=True)
    lcp2 = lib.sa_lcp(t, sa, isa)
    sa, lcp, lcp2 = sa.cpu().numpy(), lcp.cpu().numpy(), lcp2.cpu().numpy()
    assert np.array_equal(lcp, lcp2)
    for s, txt in enumerate(texts):
        lo, hi = off[s], off[s + 1]
        want_sa = oracle.suffix_array(txt)
        assert np.array_equal(sa[lo:hi] - lo, want_sa), f"set {s}"
        assert np.array_equal(lcp[lo:hi], oracle.lcp_array(txt, want_sa)), f"set {s} lcp"


def test_lcp_reports_device_failures(lib):
    """sa_lcp is asynchronous: a bad byte it meets is left in lcp[0] as the negative status,
    sa_lcp_status raises it, and sa_overlaps refuses an LCP array that carries it."""
    good = synth.genome_reads(5, 3000, 60, 80, err=0.01)
    t = dev(good)
    sa, isa = lib.sa_build(t)
    bad = good.copy()
    bad[100] = ord("N")
    lcp = lib.sa_lcp(dev(bad), sa, isa)
    assert int(lcp[0].item()) == lib.SA_ERR_ALPHABET
    with pytest.raises(lib.SaasmError) as e:
        lib.sa_lcp_status(lcp)
    assert e.value.code == lib.SA_ERR_ALPHABET
    with pytest.raises(lib.SaasmError) as e:
        lib.sa_overlaps(t, sa, isa, lcp, 20)
    assert e.value.code == lib.SA_ERR_ALPHABET
    ok = lib.sa_lcp(t, sa, isa, check=True)  # the same call on the good text reports nothing
    assert int(ok[0].item()) == 0


def test_one_workspace_for_the_path(lib):
    """sa_build, sa_lcp and sa_overlaps share one workspace of sa_workspace_bytes(n) bytes."""
    t = synth.genome_reads(31, 40_000, 1500, 200, err=0.005)
    need = lib.sa_workspace_bytes(t.size, int((t == ord("$")).sum()))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    sa, isa, lcp, ovl = lib.sa_path(dev(t), 25, ws=ws)
    want = oracle.suffix_array(t)
    assert np.array_equal(sa.cpu().numpy(), want)
    assert np.array_equal(lcp.cpu().numpy(), oracle.lcp_array(t, want))
    assert np.array_equal(ovl.cpu().numpy(), oracle.overlaps(t, 25))


def test_batched_graph_repeated_with_eager_work_between(lib):
    """The replayed-graph build, run several times with unrelated eager builds and
    synchronisations between the runs: every run equals the host-driven build."""
    texts, off, cat = _batched_case(5, 40)
    t = dev(cat)
    want, _ = lib.sa_build_batched(t, off, use_graph=False)
    want = want.cpu().numpy()
    other = dev(synth.genome_reads(77, 5000, 200, 100, err=0.01))
    other_want = oracle.suffix_array(other.cpu().numpy())
    for rep in range(4):
        got, isa = lib.sa_build_batched(t, off, use_graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want), f"graph run {rep}"
        assert np.array_equal(isa.cpu().numpy()[want], np.arange(cat.size)), f"graph run {rep}"
        o, _ = lib.sa_build(other)  # eager work between the replays
        torch.cuda.synchronize()
        assert np.array_equal(o.cpu().numpy(), other_want), f"eager run {rep}"


def test_batched_matches_plain_per_set(lib):
    texts, off, cat = _batched_case(9, 20, 1000, 20000)
    sa_b, _ = lib.sa_build_batched(dev(cat), off)
    sa_b = sa_b.cpu().numpy()
    for s, txt in enumerate(texts):
        sa_p, _ = run_sa(lib, txt)
        assert np.array_equal(sa_b[off[s]:off[s + 1]] - off[s], sa_p)


def test_batched_rejects_bad_offsets(lib):
    texts, off, cat = _batched_case(5, 3)
    bad = off.copy()
    bad[1] -= 1  # text 0 no longer ends with '$'
    with pytest.raises(lib.SaasmError):
        lib.sa_build_batched(dev(cat), bad)
    with pytest.raises(lib.SaasmError):
        lib.sa_build_batched(dev(cat), off[:-1])


def test_batched_seg_pack_identical(lib):
    """Packing texts into several builds (seg_pack) gives the same arrays as one build."""
    texts, off, cat = _batched_case(12, 40, 500, 8000)
    t = dev(cat)
    sa1, isa1 = lib.sa_build_batched(t, off)
    for pack in (1, 20_000, 100_000):
        sa2, isa2 = lib.sa_build_batched(t, off, tuning={"seg_pack": pack}, use_graph=(pack != 1))
        assert torch.equal(sa1, sa2) and torch.equal(isa1, isa2), pack
    assert lib.sa_build_batched_ws_bytes(cat.size, 40, {"seg_pack": 20_000}, off) < \
        lib.sa_build_batched_ws_bytes(cat.size, 40)


def test_autotune_picks_a_valid_tuning(lib, tmp_path):
    from paper_1404_3456_amd import autotune
    t = dev(synth.genome_reads(5, 30_000, 1000, 150, err=0.005))
    tu, rep = autotune.autotune(t, candidates=[(8, 512, 16), (9, 256, 16)], reps=1,
                                cache_path=str(tmp_path / "cache.json"))
    assert rep["cached"] is False and len(rep["tried"]) == 2
    tu2, rep2 = autotune.autotune(t, cache_path=str(tmp_path / "cache.json"))
    assert rep2["cached"] is True and tu2 == tu
    sa, _ = lib.sa_build(t, tuning=tu)
    assert np.array_equal(sa.cpu().numpy(), oracle.suffix_array(t.cpu().numpy()))


# ---- pattern lookup ------------------------------------------------------------------------

def run_lookup(lib, text, patterns):
    t = dev(text)
    sa, _ = lib.sa_build(t)
    got = lib.sa_lookup(t, sa, patterns)
    torch.cuda.synchronize()
    return got.cpu().numpy().astype(np.int64)


def test_lookup_small_workload(lib):
    r = synth.small_plain()
    pats = synth.lookup_patterns(r.text, 2000, 0, 0, 80)
    assert np.array_equal(run_lookup(lib, r.text, pats), oracle.lookup(r.text, pats))


def test_lookup_long_and_edge_patterns(lib):
    """Patterns across several 32-base windows, whole reads, reads plus one base, patterns
    longer than any read, the empty pattern, and texts with empty reads."""
    text = synth.genome_reads(5, 3000, 120, 150, err=0.002)
    tb = bytes(text)
    reads = [x for x in tb.split(b"$")[:-1]]
    pats = [b"", b"A", b"T" * 40] + reads[:20] + [x + b"A" for x in reads[:10]]
    pats += [tb[p:p + L].split(b"$")[0] for p in range(0, 2000, 37) for L in (31, 32, 33, 64, 65, 149)]
    pats += [reads[0] * 2, b"ACGT" * 50]
    assert np.array_equal(run_lookup(lib, text, pats), oracle.lookup(text, pats))
    p2 = [b"", b"A", b"AA", b"C", b"A" * 36, b"A" * 2999, b"A" * 3001, b"ACG" * 40, b"GATTACA",
          b"ACGTACGT", b"T"]
    for name in sorted(EDGE):
        t = np.frombuffer(EDGE[name], dtype=np.uint8).copy()
        assert np.array_equal(run_lookup(lib, t, p2), oracle.lookup(t, p2)), name


@pytest.mark.parametrize("seed", range(3))
def test_lookup_ragged_random(lib, seed):
    text = synth.random_dna_reads(40 + seed, 500, 0, 90, allow_empty=True)
    pats = synth.lookup_patterns(text, 1500, seed + 1, 0, 40)
    assert np.array_equal(run_lookup(lib, text, pats), oracle.lookup(text, pats))


def test_lookup_rejects_bad_patterns(lib):
    text = synth.random_dna_reads(3, 20, 5, 30)
    t = dev(text)
    sa, _ = lib.sa_build(t)
    with pytest.raises(lib.SaasmError) as e:
        lib.sa_lookup(t, sa, [b"ACGT", b"ACNT"])
    assert e.value.code == lib.SA_ERR_ALPHABET
    buf = dev(np.frombuffer(b"ACGTACGT", dtype=np.uint8).copy())
    off = dev(np.array([0, 5, 3], dtype=np.int64))  # decreasing offsets
    with pytest.raises(lib.SaasmError) as e:
        lib.sa_lookup(t, sa, (buf, off))
    assert e.value.code == lib.SA_ERR_INVALID


# ---- cut-and-continue reconstruction over the GPU-built index ------------------------------

@pytest.mark.parametrize("seed", range(3))
def test_reconstruct_vs_oracle(lib, seed):
    from oracle import recon
    _, seq, frags = synth.two_cuttings(seed, 20_000, 100, min_gap=16)
    got = lib.sa_reconstruct(synth.text_from_strings(frags))
    assert got == recon.reconstruct(frags) and got[0] == seq
    _, _, frags = synth.two_cuttings(seed, 3000, 50)  # short pieces: several answers
    assert lib.sa_reconstruct(synth.text_from_strings(frags)) == recon.reconstruct(frags)


def test_reconstruct_backtracking_and_unsolvable(lib):
    assert lib.sa_reconstruct(synth.text_from_strings([b"AC", b"ACGT", b"ACA", b"CGT"])) == \
        (b"ACACGT", [0, 2, 1, 3])
    assert lib.sa_reconstruct(synth.text_from_strings([b"AC", b"GT", b"TT"])) is None


def test_reconstruct_large_ground_truth(lib):
    """2 Mbp cut twice into ~8,000 fragments: the original sequence comes back, and the
    placement order tiles it with both cuttings."""
    _, seq, frags = synth.two_cuttings(7, 2_000_000, 500, min_gap=32)
    rs, order = lib.sa_reconstruct(synth.text_from_strings(frags))
    assert rs == seq and sorted(order) == list(range(len(frags)))
    e = [0, 0]
    for f in order:
        c = 0 if e[0] <= e[1] else 1
        assert rs[e[c]:e[c] + len(frags[f])] == frags[f]
        e[c] += len(frags[f])
    assert e == [len(seq), len(seq)]


# ---- overlaps on both strands --------------------------------------------------------------

def test_revcomp_text_layout(lib):
    text = synth.random_dna_reads(80, 50, 0, 40, allow_empty=True)
    t2, m = lib.sa_revcomp_text(dev(text))
    comp = np.arange(256, dtype=np.uint8)
    for x, y in (("A", "T"), ("C", "G"), ("G", "C"), ("T", "A")):
        comp[ord(x)] = ord(y)
    want = np.concatenate([text, comp[text[:-1][::-1]], np.array([ord("$")], dtype=np.uint8)])
    assert np.array_equal(t2.cpu().numpy(), want) and m == int((text == ord("$")).sum())


@pytest.mark.parametrize("case", ["strand_reads", "ragged", "edge"])
def test_overlaps_rc_vs_oracle(lib, case):
    if case == "strand_reads":
        texts = [(synth.strand_reads(1, 20_000, 400, 200)[0], 30)]
    elif case == "ragged":
        texts = [(synth.random_dna_reads(90 + s, 400, 0, 120, allow_empty=True), 8) for s in range(2)]
    else:
        texts = [(np.frombuffer(EDGE[k], dtype=np.uint8).copy(), 1) for k in sorted(EDGE)]
    for text, ml in texts:
        got = lib.sa_overlaps_rc(dev(text), ml).cpu().numpy()
        assert np.array_equal(got, oracle.overlaps_rc(text, ml)), (case, text.size)


def _rc_rows_of(reads, a, min_len):
    """Every row with read a first, from the three-orientation definition written out with
    prefix hashing of its own (no suffix array and none of the oracle's code): for each way the
    reads can meet, the longest l >= min_len with the last l bases of A equal to the first l of
    B, found by looking up each suffix start of A among the min_len-base prefixes of B."""
    comp = bytes.maketrans(b"ACGT", b"TGCA")

    def rc(x):
        return x.translate(comp)[::-1]

    pref = [{}, {}]  # strand-0/2 B is a read, strand-1 B is a read's reverse complement
    for b, x in enumerate(reads):
        if len(x) >= min_len:
            pref[0].setdefault(x[:min_len], []).append(b)
            pref[1].setdefault(rc(x)[:min_len], []).append(b)
    rows = {}
    for o, A, table, flip in ((0, reads[a], pref[0], False), (1, reads[a], pref[1], True),
                              (2, rc(reads[a]), pref[0], False)):
        for start in range(0, len(A) - min_len + 1):
            l = len(A) - start
            for b in table.get(A[start:start + min_len], ()):
                if b == a:
                    continue
                B = rc(reads[b]) if flip else reads[b]
                if l <= len(B) and A[start:] == B[:l] and (b, o) not in rows:
                    rows[(b, o)] = l  # start ascending: the first match is the longest
    return sorted([a, b, o, l] for (b, o), l in rows.items())


def test_overlaps_rc_sampled_large(lib):
    """A 10 M-character sample of the plain large workload (doubled to 20 M): all rows against
    the oracle, and the rows of 30 sampled reads against the three-orientation definition
    checked directly (independent of the doubled-text reduction both sides use)."""
    r = synth.large_plain(scale=0.2)
    got = lib.sa_overlaps_rc(dev(r.text), r.min_len).cpu().numpy()
    want = oracle.overlaps_rc(r.text, r.min_len)
    assert got.shape[0] > 1000 and np.array_equal(got, want)
    reads = bytes(r.text).split(b"$")[:-1]
    rng = np.random.default_rng(17)
    for a in sorted(rng.choice(len(reads), size=30, replace=False)):
        lo, hi = np.searchsorted(got[:, 0], [a, a + 1])
        mine = got[lo:hi].tolist()
        assert mine == _rc_rows_of(reads, int(a), r.min_len), f"read {a}"


def stem_family_text(seed):
    """40 reads of 360 bases: a 60-base stem shared by all, then 8 families of 5 reads sharing
    100 more bases, then a random 200-base tail each.  After the first round (29 bases) and the
    next (58) the stem still holds groups of 40; from 116 bases on no group has more than 5."""
    rng = np.random.default_rng([synth.SEED_BASE, 700, seed])
    bases = np.frombuffer(b"ACGT", dtype=np.uint8)
    stem = rng.choice(bases, 60)
    reads = []
    for _ in range(8):
        fam = rng.choice(bases, 100)
        for _ in range(5):
            reads.append(np.concatenate([stem, fam, rng.choice(bases, 200)]).tobytes().decode())
    return synth.text_from_strings(reads)


@pytest.mark.parametrize("seed", range(3))
def test_build_switches_from_radix_rounds_to_run_sort(lib, seed):
    """Rounds whose groups exceed 32 members sort by radix passes; once every group is small
    the rounds sort group by group.  A build that goes through both must still give the
    oracle's arrays, and the timing records show that both sorts did work."""
    text = stem_family_text(seed)
    n = text.size
    tuning = {"digit_bits": 9, "block_threads": 512, "items_per_thread": 16}
    lib.sa_timing_reset()
    lib.sa_timing_enable(True)
    try:
        sa, isa, lcp, ovl = run_all(lib, text, 40, tuning=tuning)
    finally:
        lib.sa_timing_enable(False)
    want = oracle.suffix_array(text)
    assert np.array_equal(sa, want)
    assert np.array_equal(isa[want], np.arange(n))
    assert np.array_equal(lcp, oracle.lcp_array(text, want))
    assert np.array_equal(ovl, oracle.overlaps(text, 40))
    _, _, radix_bytes = lib.sa_timing_get("radix_pass")
    _, _, runs_bytes = lib.sa_timing_get("keyruns")
    first_round = 7 * n * 24.0  # 63-bit first-round keys, 9-bit digits, 24 B per item
    assert radix_bytes > first_round, "no doubling round sorted by radix passes"
    assert runs_bytes > 0, "no doubling round sorted group by group"


def mixed_groups_text(seed):
    """Error-free reads of a random genome at ~10x (groups of about ten members after the first
    round, all small) plus 60 copies of one 600-base tandem read ((AC)^150 then (AGT)^100) and
    40 reads cut from a long run of a 7-base unit: the repeat suffixes stay in groups of 40 to
    several hundred members through every round, beside the many small groups."""
    rng = np.random.default_rng([synth.SEED_BASE, 701, seed])
    genome = rng.choice(np.frombuffer(b"ACGT", dtype=np.uint8), 30_000).tobytes().decode()
    reads = []
    for _ in range(1200):
        s0 = int(rng.integers(0, len(genome) - 250))
        reads.append(genome[s0:s0 + 250])
    tandem = "AC" * 150 + "AGT" * 100
    reads += [tandem] * 60
    unit = "".join(rng.choice(list("ACGT"), 7))
    long_run = unit * 400
    for _ in range(40):
        s0 = int(rng.integers(0, 7 * 300))
        reads.append(long_run[s0:s0 + 500])
    order = rng.permutation(len(reads))
    return synth.text_from_strings([reads[k] for k in order])


@pytest.mark.parametrize("seed", range(3))
def test_mixed_group_sizes_every_round(lib, seed):
    """Rounds with groups of more than 32 members beside many of at most 32: the small ones are
    sorted run by run, only the large groups' items go through the radix passes, and the build
    equals the oracle (SA, LCP, overlaps).  The timing records show both sorts working in the
    doubling rounds, over fewer radix items than active items."""
    text = mixed_groups_text(seed)
    n = text.size
    lib.sa_timing_reset()
    lib.sa_timing_enable(True)
    try:
        sa, isa, lcp, ovl = run_all(lib, text, 30)
    finally:
        lib.sa_timing_enable(False)
    want = oracle.suffix_array(text)
    assert np.array_equal(sa, want)
    assert np.array_equal(isa[want], np.arange(n))
    assert np.array_equal(lcp, oracle.lcp_array(text, want))
    assert np.array_equal(ovl, oracle.overlaps(text, 30))
    big_items = lib.sa_timing_items("keybuild")     # large-group items taken out, all rounds
    run_items = lib.sa_timing_items("keyruns")      # active items of the same rounds
    assert big_items > 0, "no large group reached the radix passes"
    assert run_items > big_items, "the small groups were not sorted run by run"


# ---- the weighted overlap graph's maximal path over GPU-built overlaps (Sec. III) ------------

@pytest.mark.parametrize("seed", range(4))
def test_overlap_path_from_gpu_overlaps(lib, seed):
    """Seven to nine reads of a short genome: the overlaps built on the GPU, the exact path
    search over them; its weight is the exhaustive maximum over the oracle's overlaps and the
    merge along it is the oracle's merge."""
    from oracle import path as opath
    m = 7 + seed % 3
    t = synth.genome_reads(500 + seed, 600, m, 150, err=0.0)
    sa, isa, lcp, ovl = run_all(lib, t, 10)
    want = oracle.overlaps(t, 10)
    assert np.array_equal(ovl.reshape(-1, 3), want)
    order, weight, rs = lib.sa_overlap_path(t, ovl)
    w = opath.weights(want)
    frags = bytes(t).split(b"$")[:-1]
    assert sorted(order) == list(range(m))
    assert weight == opath.path_weight(order, w) == opath.best_weight_exhaustive(m, w)
    assert rs == opath.merge(frags, order, w)


def test_overlap_path_greedy_on_small_workload(lib):
    """The 400-read small workload: the greedy rule over the GPU-built overlaps takes the
    oracle's steps (same order, weight and superstring)."""
    from oracle import path as opath
    r = synth.small_plain()
    sa, isa, lcp, ovl = run_all(lib, r.text, r.min_len)
    want = oracle.overlaps(r.text, r.min_len)
    assert np.array_equal(ovl.reshape(-1, 3), want)
    order, weight, rs = lib.sa_overlap_path(r.text, ovl, exact_max_m=0)
    w = opath.weights(want)
    assert order == opath.greedy_path(r.m, w)
    assert weight == opath.path_weight(order, w)
    frags = bytes(r.text).split(b"$")[:-1]
    assert rs == opath.merge(frags, order, w)
