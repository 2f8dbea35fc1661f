"""Pins for the CPU oracle (no GPU).

The oracle is only trusted because of these tests: brute force on tiny inputs, the paper's
worked example (Sec. III), closed forms, positional ground truth and invariants.  The last
group plants a mistake in a copy of the oracle's C source and checks that some pin fails.
"""
import itertools
import os
import re
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1404_3456_amd import synth
from tests import checks

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.txt")


def tiny_texts(max_len=7, max_reads=3, alphabet="ACGT"):
    """Every text of at most max_len symbols over alphabet + '$' that ends with '$' and has
    at most max_reads separators (empty reads included)."""
    out = []
    for L in range(0, max_len):
        for body in itertools.product(alphabet + "$", repeat=L):
            s = "".join(body) + "$"
            if s.count("$") <= max_reads:
                out.append(s.encode())
    return out


TINY = tiny_texts()


def test_tiny_set_size():
    assert len(TINY) > 10000
    assert b"$" in TINY and b"$$" in TINY and b"ACGTAC$" in TINY


def _sa_lcp_match(lib_sa, lib_lcp, t):
    sa = list(lib_sa(t))
    if sa != brute.suffix_array(t):
        return False
    return list(lib_lcp(t, np.asarray(sa, dtype=np.int32))) == brute.lcp_array(t, sa)


def test_sa_lcp_exhaustive_tiny():
    for t in TINY:
        assert _sa_lcp_match(oracle.suffix_array, oracle.lcp_array, t), t


def test_overlaps_exhaustive_tiny():
    for t in TINY:
        for ml in (1, 2):
            want = [list(x) for x in brute.overlaps(t, ml)]
            assert oracle.overlaps_brute(t, ml).tolist() == want, (t, ml)
            assert oracle.overlaps(t, ml).tolist() == want, (t, ml)


@pytest.mark.parametrize("seed", range(12))
def test_random_small_vs_brute(seed):
    rng = np.random.default_rng(seed)
    alphabet = [b"ACGT", b"AC", b"A", b"ACG"][seed % 4]
    t = synth.random_dna_reads(seed, int(rng.integers(1, 12)), 0, 20, alphabet=alphabet,
                               allow_empty=True).tobytes()
    assert _sa_lcp_match(oracle.suffix_array, oracle.lcp_array, t)
    for ml in (1, 3):
        want = [list(x) for x in brute.overlaps(t, ml)]
        assert oracle.overlaps_brute(t, ml).tolist() == want
        assert oracle.overlaps(t, ml).tolist() == want


def test_overlapping_reads_vs_brute():
    for seed in range(6):
        t = synth.genome_reads(seed, 60, 12, 15, err=0.02, alphabet_size=2 + seed % 3).tobytes()
        assert _sa_lcp_match(oracle.suffix_array, oracle.lcp_array, t)
        want = [list(x) for x in brute.overlaps(t, 4)]
        assert oracle.overlaps(t, 4).tolist() == want


# ---- the paper's worked example (Sec. III) -------------------------------------------------

def _golden():
    d = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            d[k.strip()] = v.split()
    return d["fragments"], d["path"], d["superstring"][0]


def _weights(frags, ovl_fn):
    t = synth.text_from_strings(frags)
    w = {}
    for a, b, l in ovl_fn(t, 1).tolist():
        w[(a, b)] = l
    return w


def _merge(frags, order, w):
    s = frags[order[0]]
    for x, y in zip(order, order[1:]):
        s += frags[y][w.get((x, y), 0):]
    return s


def check_worked_example(ovl_fn):
    frags, path, superstring = _golden()
    w = _weights(frags, ovl_fn)
    order = [frags.index(p) for p in path]
    best = max(itertools.permutations(range(len(frags))),
               key=lambda o: sum(w.get((x, y), 0) for x, y in zip(o, o[1:])))
    scores = sorted((sum(w.get((x, y), 0) for x, y in zip(o, o[1:])), o)
                    for o in itertools.permutations(range(len(frags))))
    unique_max = scores[-1][0] > scores[-2][0]
    return (list(best) == order and unique_max and _merge(frags, order, w) == superstring)


def test_worked_example_path_and_superstring():
    """Longest overlaps reproduce the paper's maximal Hamiltonian path (unique maximum over all
    120 orders) and, merged along it, the paper's superstring."""
    assert check_worked_example(oracle.overlaps)
    assert check_worked_example(oracle.overlaps_brute)
    frags, path, _ = _golden()
    w = _weights(frags, oracle.overlaps)
    order = [frags.index(p) for p in path]
    assert [w[(x, y)] for x, y in zip(order, order[1:])] == [2, 7, 4, 2]


# ---- closed forms ------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 2, 6, 40])
def test_single_homopolymer_closed_form(k):
    t = b"A" * k + b"$"
    sa = oracle.suffix_array(t)
    assert sa.tolist() == list(range(k, -1, -1))
    lcp = oracle.lcp_array(t, sa)
    assert lcp.tolist() == [0, 0] + list(range(1, k))
    assert oracle.overlaps(t, 1).shape[0] == 0


@pytest.mark.parametrize("x", [b"ACGTTGCA", b"AAAA", b"GATTACA"])
def test_identical_reads_closed_form(x):
    t = x + b"$" + x + b"$"
    n = len(t)
    sa = oracle.suffix_array(t)
    lcp = oracle.lcp_array(t, sa)
    isa = checks.isa_of(sa)
    L = len(x)
    for p in range(L + 1):           # suffix of read 0 at offset p, same suffix of read 1
        i0, i1 = isa[p], isa[p + L + 1]
        assert i1 == i0 + 1
        assert lcp[i1] == L - p
    assert oracle.overlaps(t, 1).tolist() == [[0, 1, L], [1, 0, L]]
    assert n == 2 * L + 2


def test_single_read_textbook_sa():
    x = b"GATTACAGATTACA"
    t = x + b"$"
    sa = oracle.suffix_array(t)
    # textbook SA of x$ with $ smallest: sort suffixes as Python bytes with '$' < letters
    want = sorted(range(len(t)), key=lambda p: t[p:])
    assert sa.tolist() == want


# ---- positional ground truth and invariants at the small plain workload -----------------

@pytest.fixture(scope="module")
def small():
    r = synth.small_plain()
    sa = oracle.suffix_array(r.text)
    lcp = oracle.lcp_array(r.text, sa)
    return r, sa, lcp


def test_small_positional_ground_truth(small):
    r, _, _ = small
    want = checks.positional_overlaps(r.starts, 200, r.min_len)
    got = oracle.overlaps(r.text, r.min_len)
    assert np.array_equal(got, want)
    assert np.array_equal(oracle.overlaps_brute(r.text, r.min_len), want)


def test_ragged_positional_ground_truth():
    """The vectorised positional truth for reads of mixed lengths (equal starts, contained
    reads, a read ending where another ends) equals the brute-force overlaps and, for equal
    lengths, the per-read positional truth."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([synth.SEED_BASE, 77])))
    g = 3000
    genome = synth.random_genome(rng, g)
    for L_lo, L_hi in ((60, 60), (20, 90)):
        lengths = rng.integers(L_lo, L_hi + 1, size=120)
        starts = rng.integers(0, g - lengths + 1)
        starts[5] = starts[6]            # equal starts
        starts[7], lengths[7] = starts[8], lengths[8]  # identical reads
        text = synth.layout_text(genome, starts, lengths, 0.0, None)
        want = checks.positional_overlaps_ragged(starts, lengths, 15)
        assert np.array_equal(oracle.overlaps_brute(text, 15), want), (L_lo, L_hi)
        if L_lo == L_hi:
            assert np.array_equal(checks.positional_overlaps(starts, L_lo, 15), want)


def test_small_invariants(small):
    r, sa, lcp = small
    checks.assert_sa_basic(r.text, sa)
    idx = np.arange(r.n, dtype=np.int64)
    bad, first = oracle.check_adjacent(r.text, sa, lcp, idx)
    assert bad == 0, first
    checks.assert_kasai_property(r.text, sa, lcp)
    checks.assert_lcp_bounds(r.text, sa, lcp)


def test_small_overlaps_reverse_lookup(small):
    r, _, _ = small
    fwd = oracle.overlaps(r.text, r.min_len)
    rev = oracle.overlaps(checks.reversed_reads_text(r.text), r.min_len)
    assert np.array_equal(checks.swap_pairs(fwd), rev)
    checks.assert_overlaps_valid(r.text, fwd[:200], r.min_len)


def test_ragged_invariants():
    t = synth.random_dna_reads(99, 300, 0, 60, alphabet=b"AC", allow_empty=True)
    sa = oracle.suffix_array(t)
    lcp = oracle.lcp_array(t, sa)
    checks.assert_sa_basic(t, sa)
    bad, _ = oracle.check_adjacent(t, sa, lcp, np.arange(t.size))
    assert bad == 0
    checks.assert_kasai_property(t, sa, lcp)
    checks.assert_lcp_bounds(t, sa, lcp)
    ovl = oracle.overlaps(t, 5)
    checks.assert_overlaps_valid(t, ovl, 5)
    assert np.array_equal(ovl, oracle.overlaps_brute(t, 5))
    rev = oracle.overlaps(checks.reversed_reads_text(t), 5)
    assert np.array_equal(checks.swap_pairs(ovl), rev)


def test_rejects_bad_text():
    with pytest.raises(ValueError):
        oracle.suffix_array(b"ACGT")
    with pytest.raises(ValueError):
        oracle.suffix_array(b"")


# ---- pattern lookup -------------------------------------------------------------------------

LOOKUP_PATTERNS = [b""] + [bytes(x) for L in (1, 2, 3) for x in itertools.product(b"ACGT", repeat=L)]


def _lookup_matches_brute(lookup_fn, t, patterns):
    got = lookup_fn(t, patterns).tolist()
    return got == [list(brute.lookup(t, p)) for p in patterns]


def test_lookup_vs_brute_tiny():
    """Every pattern of length <= 3 on a sample of the tiny texts, against the SA-based literal
    definition of the interval."""
    for t in TINY[::13]:
        assert _lookup_matches_brute(oracle.lookup, t, LOOKUP_PATTERNS), t


@pytest.mark.parametrize("k", [1, 3, 9])
def test_lookup_homopolymer_closed_form(k):
    """Text A^k$: the suffixes are $, A$, ..., A^k$ in that order, so A^j (1 <= j <= k) starts
    exactly the last k-j+1 of them: [j, k+1); A^(k+1) starts none and sorts after all."""
    t = b"A" * k + b"$"
    pats = [b"A" * j for j in range(1, k + 2)] + [b"C", b""]
    got = oracle.lookup(t, pats).tolist()
    want = [[j, k + 1] for j in range(1, k + 1)] + [[k + 1, k + 1], [k + 1, k + 1], [0, k + 1]]
    assert got == want


@pytest.mark.parametrize("seed", [0, 1])
def test_lookup_interval_invariants(seed):
    """On random reads: the interval width is the number of occurrences (counted with
    str.find), every suffix inside starts with the pattern, and its neighbours do not."""
    rng = np.random.default_rng(seed)
    reads = ["".join(rng.choice(list("ACGT"), size=int(rng.integers(0, 30)))) for _ in range(40)]
    t = synth.text_from_strings(reads)
    sa = oracle.suffix_array(t)
    tb = bytes(t)
    pats = [tb[p:p + L] for p, L in zip(rng.integers(0, len(tb) - 8, 60), rng.integers(1, 8, 60))]
    pats = [p for p in pats if b"$" not in p] + [b"ACGTACGTAC", b"TTTTT"]
    for p, (lo, hi) in zip(pats, oracle.lookup(t, pats).tolist()):
        occ, i = 0, tb.find(p)
        while i >= 0:
            occ, i = occ + 1, tb.find(p, i + 1)
        assert hi - lo == occ
        assert all(tb[q:q + len(p)] == p for q in sa[lo:hi])
        if lo > 0:
            assert tb[sa[lo - 1]:sa[lo - 1] + len(p)] != p
        if hi < len(tb):
            assert tb[sa[hi]:sa[hi] + len(p)] != p


def test_lookup_worked_example_superstring():
    """Sec. III worked example: the printed superstring contains every fragment, and merging
    along the printed path places them in path order (first occurrences increase)."""
    frags, path, superstring = _golden()
    t = superstring.encode() + b"$"
    res = oracle.lookup(t, [p.encode() for p in path]).tolist()
    assert all(hi - lo >= 1 for lo, hi in res)
    first = [superstring.find(p) for p in path]
    assert first == sorted(first) and first[0] == 0


def test_lookup_rejects_separator_in_pattern():
    with pytest.raises(ValueError):
        oracle.lookup(b"ACGT$", [b"A$"])


# ---- overlaps on both strands ----------------------------------------------------------------

def test_overlaps_rc_vs_brute():
    for t in TINY[::23]:
        for ml in (1, 2):
            assert oracle.overlaps_rc(t, ml).tolist() == brute.overlaps_rc(t, ml), (t, ml)
    for seed in range(3):
        t = bytes(synth.random_dna_reads(60 + seed, 25, 1, 14))
        assert oracle.overlaps_rc(t, 3).tolist() == brute.overlaps_rc(t, 3)


def test_overlaps_rc_strand_symmetry():
    """Ends meeting (strand 1) and starts meeting (strand 2) are symmetric in a and b: the last
    l bases of a equal the first l of revcomp(b) exactly when the same holds with a and b
    swapped, and likewise for revcomp(a) before b."""
    t = bytes(synth.random_dna_reads(70, 300, 20, 80))
    rows = oracle.overlaps_rc(t, 5).tolist()
    for o in (1, 2):
        s = {(a, b, l) for a, b, oo, l in rows if oo == o}
        assert s and s == {(b, a, l) for a, b, l in s}, o


def test_overlaps_rc_positional_ground_truth():
    """Error-free reads from both strands of a random genome: every overlap is the one their
    genome positions and orientations imply."""
    text, starts, strands = synth.strand_reads(0, 20_000, 400, 200)
    got = oracle.overlaps_rc(text, 30)
    want = checks.positional_overlaps_rc(starts, strands, 200, 30)
    assert np.array_equal(got, want)
    assert (got[:, 2] == 1).sum() > 100 and (got[:, 2] == 2).sum() > 100


# ---- planted mistakes: each mutant of the C oracle must fail some pin --------------------

MUTANTS = {
    # separators ordered against read order
    "sep_order": (r"return \(p < q\) \? -1 : 1; /\* separator", "return (p < q) ? 1 : -1; /* separator"),
    # LCP runs through separators as if they were equal symbols
    "lcp_through_sep": (r"while \(t\[p \+ k\] == t\[q \+ k\] && t\[p \+ k\] != SEPB\) \+\+k;\n        lcp\[i\]",
                        "while (t[p + k] == t[q + k] && p + k < n - 1 && q + k < n - 1) ++k;\n        lcp[i]"),
    # shortest instead of longest overlap (brute force)
    "brute_shortest": (r"for \(int64_t l = top; l >= min_len; --l\)",
                       "for (int64_t l = min_len; l <= top; ++l)"),
    # containment (l = |a|) never tried by the indexed search
    "indexed_no_containment": (r"for \(int64_t o = 0; o \+ min_len <= la; \+\+o\)",
                               "for (int64_t o = 1; o + min_len <= la; ++o)"),
    # off by one at the minimum length
    "indexed_min_len_off_by_one": (r"for \(int64_t o = 0; o \+ min_len <= la; \+\+o\)",
                                   "for (int64_t o = 0; o + min_len < la; ++o)"),
    # a suffix that ends at its separator counted above the pattern
    "lookup_sep_above": (r"if \(x == SEPB\) return -1;  /\* the suffix ends first",
                         "if (x == SEPB) return 1;  /* the suffix ends first"),
    # suffixes that start with the pattern counted below it
    "lookup_prefix_below": (r"if \(c < 0\) \+\+below;", "if (c <= 0) ++below;"),
}


def _pins_pass(lib_dir):
    """Run a reduced pin suite against an oracle built in lib_dir; True when all pass."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "oracle_mut", os.path.join(lib_dir, "__init__.py"), submodule_search_locations=[lib_dir])
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    try:
        for t in TINY[::7]:
            if not _sa_lcp_match(mod.suffix_array, mod.lcp_array, t):
                return False
            for ml in (1, 2):
                want = [list(x) for x in brute.overlaps(t, ml)]
                if mod.overlaps_brute(t, ml).tolist() != want or mod.overlaps(t, ml).tolist() != want:
                    return False
        if not check_worked_example(mod.overlaps) or not check_worked_example(mod.overlaps_brute):
            return False
        for t in TINY[::97]:
            if not _lookup_matches_brute(mod.lookup, t, LOOKUP_PATTERNS[:21]):
                return False
        return True
    except Exception:
        return False


@pytest.mark.parametrize("name", ["none"] + sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    src_dir = os.path.dirname(oracle.__file__)
    d = tmp_path / "oracle_mut"
    d.mkdir()
    shutil.copy(os.path.join(src_dir, "__init__.py"), d / "__init__.py")
    src = open(os.path.join(src_dir, "saoracle.c")).read()
    if name != "none":
        pat, rep = MUTANTS[name]
        src2, k = re.subn(pat, rep, src)
        assert k >= 1, f"mutation {name} did not apply"
        src = src2
    (d / "saoracle.c").write_text(src)
    ok = _pins_pass(str(d))
    if name == "none":
        assert ok, "unmutated oracle must pass its pins"
    else:
        assert not ok, f"planted mistake {name} was not caught by any pin"


# ---- the merge path of the oracle's parallel sort, and the exhaustive full-size check -------

def _merge_path_texts():
    return [
        synth.random_dna_reads(77, 90, 20, 120, allow_empty=True),
        synth.genome_reads(78, 1500, 60, 90, err=0.0),     # heavy overlap: long equal prefixes
        synth.genome_reads(79, 900, 40, 150, err=0.01, alphabet_size=2),
        np.frombuffer(b"A" * 3000 + b"$" + b"AC" * 1000 + b"$" + b"A" * 2500 + b"$",
                      dtype=np.uint8).copy(),
    ]


@pytest.mark.parametrize("nthreads", [2, 3, 8])
def test_sa_merge_path_vs_brute(nthreads):
    """Above 4096 characters the oracle sorts per-thread chunks and merges them; that order
    must still be the literal definition's."""
    for t in _merge_path_texts():
        assert t.size > 4096
        want = np.array(brute.suffix_array(t.tobytes()), dtype=np.int32)
        assert np.array_equal(oracle.suffix_array(t, nthreads=nthreads), want)


def test_check_all_agrees_with_bytewise_check():
    """check_all (whole words skipped while equal and separator-free) fails exactly the
    indices the byte-by-byte check_adjacent fails, on correct arrays and on planted errors:
    swapped neighbours, a moved entry, an LCP off by one either way, a repeated entry."""
    rng = np.random.default_rng(3)
    for t in _merge_path_texts() + [np.frombuffer(s, dtype=np.uint8).copy() for s in TINY[::97]]:
        n = t.size
        sa = oracle.suffix_array(t)
        lcp = oracle.lcp_array(t, sa)
        every = np.arange(1, n, dtype=np.int64)
        assert oracle.check_all(t, sa, lcp) == (0, -1)
        assert oracle.check_adjacent(t, sa, lcp, every) == (0, -1)
        if n < 3:
            continue
        for trial in range(6):
            s2, l2 = sa.copy(), lcp.copy()
            i = int(rng.integers(1, n - 1))
            if trial == 0:
                s2[i], s2[i + 1] = s2[i + 1], s2[i]
            elif trial == 1:
                j = int(rng.integers(0, n))
                s2 = np.insert(np.delete(s2, i), j, s2[i])
            elif trial == 2:
                l2[i] += 1
            elif trial == 3:
                l2[i] -= 1
            elif trial == 4:
                s2[i] = s2[i - 1]
            else:
                s2 = s2[::-1].copy()
            got = oracle.check_all(t, s2, l2)
            want = oracle.check_adjacent(t, s2, l2, every)
            assert got == want, (trial, got, want)
            if trial != 1 or not np.array_equal(s2, sa):
                assert got[0] > 0 or (trial == 1 and np.array_equal(s2, sa)), trial
