"""GPU parity of the skew (DC3) build: sa_build_dc3, called through the C ABI, against the
oracle's suffix array on the same seeded inputs (exact), and at full workload sizes against
what the oracle checks at any size (permutation, every adjacent pair's order and LCP)."""
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


def run_dc3(lib, text, tuning=None):
    sa, isa, levels = lib.sa_build_dc3(dev(text), tuning=tuning, return_levels=True)
    torch.cuda.synchronize()
    return sa.cpu().numpy(), isa.cpu().numpy(), levels


def assert_dc3(lib, text, tuning=None, label=""):
    sa, isa, levels = run_dc3(lib, text, tuning)
    want = oracle.suffix_array(text)
    assert np.array_equal(sa, want), f"SA mismatch {label}"
    assert np.array_equal(isa[sa], np.arange(text.size)), f"ISA mismatch {label}"
    return levels


def as_text(b):
    return np.frombuffer(b, dtype=np.uint8).copy()


def test_dc3_tiny_exhaustive(lib):
    texts = []
    for L in range(0, 6):
        for body in itertools.product("ACGT$", repeat=L):
            texts.append(as_text(("".join(body) + "$").encode()))
    for t in texts:
        sa, isa, _ = run_dc3(lib, t)
        assert np.array_equal(sa, oracle.suffix_array(t)), t.tobytes()


EDGE = {
    "one_sep": b"$",
    "two_seps": b"$$",
    "three_seps": b"$$$",
    "one_base": b"A$",
    "empty_reads": b"$AC$$GT$$",
    "homopolymer_10k": b"A" * 10_000 + b"$",
    "homopolymer_10k_plus1": b"A" * 10_001 + b"$",
    "homopolymer_10k_plus2": b"A" * 10_002 + b"$",
    "two_identical": b"ACGTTGCAAC$ACGTTGCAAC$",
    "many_identical": b"GATTACA$" * 300,
    "period3_5k": b"ACG" * 1700 + b"$",
    "period2_4k": b"AC" * 2000 + b"$",
    "two_homopolymers": b"A" * 3000 + b"$" + b"A" * 2999 + b"$",
    "nested": b"ACGTACGTACGT$CGTACG$GTAC$T$",
    "all_separators": b"$" * 5000,
}


@pytest.mark.parametrize("name", sorted(EDGE))
def test_dc3_edge_cases(lib, name):
    assert_dc3(lib, as_text(EDGE[name]), label=name)


def test_dc3_recursion_depth_on_a_homopolymer(lib):
    """A^k$ needs a level per factor of 3 in k: the names of a level cover 3^(level+1)
    symbols, and only the triples that reach the separator are unique."""
    levels = assert_dc3(lib, as_text(b"A" * 6560 + b"$"), label="A^6560")
    assert 7 <= levels <= 12, levels


@pytest.mark.parametrize("seed,m,lo,hi,alpha", [
    (11, 200, 0, 50, b"ACGT"),
    (12, 400, 0, 120, b"AC"),
    (13, 2000, 1, 30, b"A"),
    (14, 50, 500, 2000, b"ACGT"),
    (15, 3000, 0, 40, b"ACG"),
])
def test_dc3_ragged_random(lib, seed, m, lo, hi, alpha):
    t = synth.random_dna_reads(seed, m, lo, hi, alphabet=alpha, allow_empty=True)
    assert_dc3(lib, t, label=f"seed{seed}")


@pytest.mark.parametrize("seed", range(4))
def test_dc3_overlapping_reads(lib, seed):
    t = synth.genome_reads(seed, 3000 + 1000 * seed, 300, 80 + 20 * seed, err=0.01 * (seed % 2),
                           alphabet_size=2 + seed % 3)
    assert_dc3(lib, t, label=f"genome{seed}")


def test_dc3_small_plain_workload(lib):
    r = synth.small_plain()
    assert assert_dc3(lib, r.text, label=r.name) > 1


@pytest.mark.parametrize("tuning", [None, {"digit_bits": 8}, {"digit_bits": 11},
                                    {"digit_bits": 4, "block_threads": 256, "items_per_thread": 8}])
def test_dc3_tunings(lib, tuning):
    t = synth.genome_reads(99, 20_000, 600, 150, err=0.005)
    assert_dc3(lib, t, tuning=tuning, label=str(tuning))


def top_level_names(text):
    """Distinct names of the top level's sample triples, counted on the CPU from the text: a
    triple that reaches a separator is a name of its own, the others are named by content."""
    n = text.size
    p = np.arange(n)
    p = p[p % 3 != 0]
    sep = text == ord("$")
    sep_pad = np.concatenate([sep, [True, True]])
    holds_sep = sep_pad[p] | sep_pad[p + 1] | sep_pad[p + 2]
    q = p[~holds_sep]
    pad = np.concatenate([text, np.zeros(2, np.uint8)]).astype(np.int64)
    trip = (pad[q] << 16) | (pad[q + 1] << 8) | pad[q + 2]
    return int(holds_sep.sum()) + np.unique(trip).size


def test_dc3_wide_names_two_sorts(lib):
    """More than 2^21 distinct names below the top level: the name triple no longer fits 64
    bits and is sorted in two radix sorts (last name, then the first two)."""
    t = synth.random_dna_reads(21, 1_200_000, 3, 6)
    k = top_level_names(t)
    assert k > (1 << 21), k
    levels = assert_dc3(lib, t, label="wide names")
    assert levels >= 2


def test_dc3_repeat_runs_identical(lib):
    t = synth.genome_reads(7, 50_000, 2000, 100, err=0.005)
    first, _, _ = run_dc3(lib, t)
    for _ in range(3):
        again, _, _ = run_dc3(lib, t)
        assert np.array_equal(first, again)


def test_dc3_rejects_bad_text(lib):
    for bad in (b"ACGT", b"ACNT$", b"acgt$"):
        with pytest.raises(lib.SaasmError):
            lib.sa_build_dc3(dev(as_text(bad)))
        torch.cuda.synchronize()


def full_dc3(lib, r):
    print(f"full-size dc3 case {r.name}: n={r.n}", flush=True)
    t = torch.from_numpy(r.text).cuda()
    sa, isa, levels = lib.sa_build_dc3(t, return_levels=True)
    sa2, _ = lib.sa_build(t, isa=False)
    same = bool(torch.equal(sa, sa2))
    del sa2
    lcp = lib.sa_lcp(t, sa, isa)
    torch.cuda.synchronize()
    sa, isa, lcp = sa.cpu().numpy(), isa.cpu().numpy(), lcp.cpu().numpy()
    del t
    checks.assert_sa_basic(r.text, sa)
    assert np.array_equal(isa[sa], np.arange(r.n, dtype=np.int32))
    bad, first = oracle.check_all(r.text, sa, lcp)
    assert bad == 0, f"{bad} bad adjacent pairs, the first at {first}"
    assert same, "the two constructions disagree"
    return levels


def test_full_dc3_plain_large(lib):
    levels = full_dc3(lib, synth.large_plain())
    assert levels > 3


def test_full_dc3_repeat_stress(lib):
    levels = full_dc3(lib, synth.repeat_stress())
    assert levels > 3
