"""Parity at full workload sizes, in the launch configuration the benchmark times.  The suffix
array and LCP are checked element by element: the SA is a permutation and every adjacent pair
of suffixes ascends with its LCP entry equal to the direct common prefix (oracle.check_all over
all n - 1 pairs), which together are the definition -- a permutation whose neighbours all ascend
is the sorted order.  Overlaps are compared whole with the oracle's exact seed-and-verify
search (or, at the largest size, with the exact positional truth of error-free reads)."""
import numpy as np
import pytest

import oracle
from paper_1404_3456_amd import synth
from tests import checks

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pkg():
    import paper_1404_3456_amd as p
    p.load()
    return p


def full_check(pkg, r):
    print(f"full-size case {r.name}: n={r.n}", flush=True)
    t = torch.from_numpy(r.text).cuda()
    sa, isa = pkg.sa_build(t)
    lcp = pkg.sa_lcp(t, sa, isa)
    ovl = pkg.sa_overlaps(t, sa, isa, lcp, r.min_len)
    torch.cuda.synchronize()
    sa, isa, lcp, ovl = sa.cpu().numpy(), isa.cpu().numpy(), lcp.cpu().numpy(), ovl.cpu().numpy()
    del t
    checks.assert_sa_basic(r.text, sa)
    assert np.array_equal(isa[sa], np.arange(r.n, dtype=np.int32))
    bad, first = oracle.check_all(r.text, sa, lcp)
    assert bad == 0, f"{bad} bad adjacent pairs, the first at {first}"
    assert lcp[0] == 0
    checks.assert_kasai_property(r.text, sa, lcp)
    want = oracle.overlaps(r.text, r.min_len)
    assert np.array_equal(ovl, want)
    return want.shape[0]


def test_full_plain_large(pkg):
    rows = full_check(pkg, synth.large_plain())
    assert rows > 100_000


def test_full_repeat_stress(pkg):
    rows = full_check(pkg, synth.repeat_stress())
    assert rows > 0


def test_full_lookup_plain_large(pkg):
    """Pattern lookup on the 50.1 M-character suffix array: sampled patterns against the
    oracle's definition over text positions."""
    r = synth.large_plain()
    print(f"full-size lookup {r.name}: n={r.n}", flush=True)
    t = torch.from_numpy(r.text).cuda()
    sa, _ = pkg.sa_build(t)
    pats = synth.lookup_patterns(r.text, 48, 3, 20, 120)
    got = pkg.sa_lookup(t, sa, pats).cpu().numpy().astype(np.int64)
    assert np.array_equal(got, oracle.lookup(r.text, pats))


def max_size_text():
    """The longest text the library accepts, n = 2^31 - 3: error-free reads of 999 bases from
    a 200 Mbp random genome (about 10.7x coverage), the last read shortened to fill n exactly.
    Returns the text and the reads' starts and lengths."""
    n = (1 << 31) - 3
    L = 999
    m_full = n // (L + 1)
    rest = n - m_full * (L + 1)
    lengths = np.full(m_full + (1 if rest else 0), L, dtype=np.int64)
    if rest:
        lengths[-1] = rest - 1
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([synth.SEED_BASE, 31])))
    g = 200_000_000
    genome = synth.random_genome(rng, g)
    starts = rng.integers(0, g - L + 1, size=lengths.size, dtype=np.int64)
    text = synth.layout_text(genome, starts, lengths, 0.0, None)
    assert text.size == n
    return text, starts, lengths


def test_full_max_size(pkg):
    """n = 2^31 - 3 (positions, ranks and counts at the edge of 32 bits): SA, ISA, LCP and
    overlaps through the C ABI, and the skew construction's SA.  SA and LCP: permutation and
    every adjacent pair's order and LCP; the skew SA equal to the checked one.  Overlaps: the
    exact positional truth of error-free reads from a random genome, and direct string checks
    of sampled rows."""
    text, starts, lengths = max_size_text()
    n = text.size
    print(f"max-size case: n={n}", flush=True)
    t = torch.from_numpy(text).cuda()
    sa, isa = pkg.sa_build(t)
    lcp = pkg.sa_lcp(t, sa, isa)
    ovl = pkg.sa_overlaps(t, sa, isa, lcp, 100)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()  # the skew build's workspace is about 72 bytes per suffix
    sa3, _, levels = pkg.sa_build_dc3(t, isa=False, return_levels=True)
    same_dc3 = bool(torch.equal(sa3, sa))
    del sa3
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(f"max-size case: GPU done (skew build: {levels} levels)", flush=True)
    sa, isa, lcp, ovl = sa.cpu().numpy(), isa.cpu().numpy(), lcp.cpu().numpy(), ovl.cpu().numpy()
    del t
    checks.assert_sa_basic(text, sa)
    assert np.array_equal(isa[sa], np.arange(n, dtype=np.int32))
    del isa
    assert same_dc3, "the skew construction differs from the doubling one"
    bad, first = oracle.check_all(text, sa, lcp)
    assert bad == 0, f"{bad} bad adjacent pairs, the first at {first}"
    assert lcp[0] == 0
    rng = np.random.default_rng(7)
    del sa, lcp
    want = checks.positional_overlaps_ragged(starts, lengths, 100)
    assert np.array_equal(ovl, want)
    rows = ovl[np.sort(rng.choice(ovl.shape[0], size=2000, replace=False))]
    checks.assert_overlaps_valid(text, rows, 100)
    print(f"max-size case: {want.shape[0]} overlap rows checked", flush=True)


def test_full_batched_256(pkg):
    """The 256-set batched workload (1.43 G characters) in one build, as the benchmark runs it:
    every set's block of the SA is a permutation of its own positions, ISA is the inverse,
    every adjacent pair inside every set ascends with its LCP equal to the direct common prefix
    (LCP 0 at set starts), and every set's overlap rows equal the oracle's overlaps of that set
    alone."""
    sets = synth.batched_sets()
    off = np.concatenate([[0], np.cumsum([s.text.size for s in sets])]).astype(np.int64)
    cat = np.concatenate([s.text for s in sets])
    n = cat.size
    print(f"full-size batched: {len(sets)} sets, n={n}", flush=True)
    t = torch.from_numpy(cat).cuda()
    sa, isa = pkg.sa_build_batched(t, off, use_graph=False)
    lcp = pkg.sa_lcp(t, sa, isa)
    ovl = pkg.sa_overlaps(t, sa, isa, lcp, 40)
    torch.cuda.synchronize()
    sa, isa, lcp, ovl = sa.cpu().numpy(), isa.cpu().numpy(), lcp.cpu().numpy(), ovl.cpu().numpy()
    del t
    assert np.all(np.bincount(sa, minlength=n) == 1), "SA is not a permutation"
    assert np.array_equal(isa[sa], np.arange(n, dtype=np.int32))
    del isa
    for s in range(len(sets)):
        lo, hi = int(off[s]), int(off[s + 1])
        blk = sa[lo:hi]
        assert blk.min() == lo and blk.max() == hi - 1, f"set {s} block"
        seps = checks.separators(sets[s].text) + lo
        assert np.array_equal(blk[: seps.size], seps), f"set {s}: separators first, in order"
        assert lcp[lo] == 0, f"set {s} first LCP"
    for s in range(len(sets)):
        lo, hi = int(off[s]), int(off[s + 1])
        bad, first = oracle.check_all(cat, sa, lcp, lo=lo + 1, hi=hi)
        assert bad == 0, f"set {s}: {bad} bad adjacent pairs, the first at {first}"
    del sa, lcp
    reads = np.array([0] + [int((s.text == ord("$")).sum()) for s in sets]).cumsum()
    set_of_read = np.repeat(np.arange(len(sets)), np.diff(reads))
    assert np.array_equal(set_of_read[ovl[:, 0]], set_of_read[ovl[:, 1]]), "rows across sets"
    for s in range(len(sets)):
        a0, a1 = np.searchsorted(ovl[:, 0], [reads[s], reads[s + 1]])
        want = oracle.overlaps(sets[s].text, 40).astype(np.int64)
        want[:, :2] += reads[s]
        assert np.array_equal(ovl[a0:a1].astype(np.int64), want), f"set {s} overlaps"
    print(f"full-size batched: {ovl.shape[0]} rows, all {len(sets)} sets against the oracle",
          flush=True)
