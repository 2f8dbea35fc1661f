"""Randomised parity sweep: many small seeded texts of mixed structure (ragged random reads,
overlapping reads with errors, tandem repeats, homopolymers, runs of empty reads, identical
reads) through both suffix-array constructions, the LCP array and the overlaps, each against
the oracle exactly.  Each case also draws a tile shape, so every tuning meets every kind of
text."""
import numpy as np
import pytest

import oracle
from paper_1404_3456_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TUNINGS = [None,
           {"digit_bits": 4, "block_threads": 256, "items_per_thread": 8},
           {"digit_bits": 8, "block_threads": 512, "items_per_thread": 16},
           {"digit_bits": 9, "block_threads": 256, "items_per_thread": 16},
           {"digit_bits": 11, "block_threads": 512, "items_per_thread": 8}]


@pytest.fixture(scope="module")
def lib():
    import paper_1404_3456_amd as pkg
    pkg.load()
    return pkg


def case_text(seed):
    """A seeded text of one of seven kinds, at most a few tens of thousands of characters."""
    rng = np.random.default_rng([synth.SEED_BASE, 500, seed])
    kind = seed % 7
    if kind == 0:
        alpha = [b"A", b"AC", b"ACG", b"ACGT"][int(rng.integers(4))]
        return synth.random_dna_reads(seed, int(rng.integers(1, 400)), 0,
                                      int(rng.integers(1, 200)), alphabet=alpha, allow_empty=True)
    if kind == 1:
        g = int(rng.integers(200, 20_000))
        return synth.genome_reads(seed, g, int(rng.integers(2, 300)),
                                  int(rng.integers(10, min(400, g))),
                                  err=float(rng.choice([0.0, 0.005, 0.05])),
                                  alphabet_size=int(rng.integers(2, 5)))
    if kind == 2:  # tandem repeats of a short unit, cut into reads
        unit = rng.choice(list(b"ACGT"), size=int(rng.integers(1, 9))).astype(np.uint8)
        body = np.tile(unit, int(rng.integers(10, 3000)))
        cuts = np.sort(rng.choice(np.arange(1, body.size), size=min(body.size - 1,
                                  int(rng.integers(0, 40))), replace=False))
        reads = np.split(body, cuts)
        return synth.text_from_strings([r.tobytes().decode() for r in reads])
    if kind == 3:  # homopolymer reads of many lengths
        lens = rng.integers(0, 300, size=int(rng.integers(1, 60)))
        base = "ACGT"[int(rng.integers(4))]
        return synth.text_from_strings([base * int(L) for L in lens])
    if kind == 4:  # runs of empty reads between short ones
        reads = []
        for _ in range(int(rng.integers(1, 200))):
            reads.append("" if rng.random() < 0.5 else
                         "".join(rng.choice(list("ACGT"), size=int(rng.integers(1, 8)))))
        return synth.text_from_strings(reads)
    if kind == 5:  # identical reads, in blocks
        r = "".join(rng.choice(list("ACGT"), size=int(rng.integers(1, 120))))
        return synth.text_from_strings([r] * int(rng.integers(2, 100)))
    # kind 6: a read set whose reads are prefixes and suffixes of one another
    s = "".join(rng.choice(list("ACGT"), size=int(rng.integers(5, 400))))
    reads = []
    for _ in range(int(rng.integers(2, 80))):
        a = int(rng.integers(0, len(s)))
        b = int(rng.integers(a, len(s) + 1))
        reads.append(s[:b] if rng.random() < 0.5 else s[a:])
    return synth.text_from_strings(reads)


@pytest.mark.parametrize("block", range(12))
def test_random_sweep(lib, block):
    for seed in range(block * 100, block * 100 + 100):
        text = case_text(seed)
        rng = np.random.default_rng([synth.SEED_BASE, 501, seed])
        tuning = TUNINGS[int(rng.integers(len(TUNINGS)))]
        min_len = int(rng.integers(1, 50))
        t = torch.from_numpy(text).cuda()
        sa, isa = lib.sa_build(t, tuning=tuning)
        sa3, isa3 = lib.sa_build_dc3(t, tuning=tuning)
        lcp = lib.sa_lcp(t, sa, isa)
        ovl = lib.sa_overlaps(t, sa, isa, lcp, min_len)
        torch.cuda.synchronize()
        want = oracle.suffix_array(text)
        label = f"seed {seed} (kind {seed % 7}, n={text.size}, tuning {tuning})"
        assert np.array_equal(sa.cpu().numpy(), want), label
        assert np.array_equal(sa3.cpu().numpy(), want), label + " dc3"
        assert np.array_equal(isa.cpu().numpy()[want], np.arange(text.size)), label
        assert np.array_equal(isa3.cpu().numpy()[want], np.arange(text.size)), label + " dc3"
        assert np.array_equal(lcp.cpu().numpy(), oracle.lcp_array(text, want)), label
        assert np.array_equal(ovl.cpu().numpy(), oracle.overlaps(text, min_len)), label
