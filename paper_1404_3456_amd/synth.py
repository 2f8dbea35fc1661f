"""Seeded synthetic shotgun-read workloads.

This module only draws genomes and reads and lays them out as one ASCII text in which every
read is followed by its own '$' separator.  It holds none of the suffix-array, LCP or overlap
arithmetic, so both the GPU library's tests and the CPU oracle's tests can take their inputs
from it without sharing any of the method.

The paper evaluates on shotgun fragments of a bacterial genome (Sec. V); that data is not
available here, so every workload below is synthetic: i.i.d. uniform A/C/G/T genomes, reads at
uniform random start positions, optional uniform substitution errors, and (for the
repeat-heavy workload) interspersed and tandem repeats written over the background.

Every generator is driven by ``numpy.random.SeedSequence(SEED_BASE + workload_index)``, with
one spawned child stream per role (genome, starts, errors, ...), so a workload is a pure
function of its parameters.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np

SEED_BASE = 14043456
SEP = ord("$")
_ASCII = np.frombuffer(b"ACGT", dtype=np.uint8)
_CHUNK_READS = 8192  # fixed chunking keeps the random draw order independent of memory


@dataclasses.dataclass
class ReadSet:
    """One text: reads r_0 $ r_1 $ ... r_{m-1} $ as ASCII bytes."""

    name: str
    text: np.ndarray          # uint8[N], ASCII 'A','C','G','T','$'
    starts: np.ndarray        # int64[m], genome start of each read (-1 if not from a genome)
    lengths: np.ndarray       # int64[m], read lengths
    min_len: int              # minimum reported overlap length
    genome_len: int
    params: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.text.size)

    @property
    def m(self) -> int:
        return int(self.lengths.size)

    def sha256(self) -> str:
        return hashlib.sha256(self.text.tobytes()).hexdigest()


def _rngs(index: int, k: int):
    ss = np.random.SeedSequence(SEED_BASE + index)
    return [np.random.Generator(np.random.PCG64(c)) for c in ss.spawn(k)]


def random_genome(rng: np.random.Generator, g: int) -> np.ndarray:
    """Codes 0..3 (A,C,G,T), i.i.d. uniform."""
    return rng.integers(0, 4, size=g, dtype=np.uint8)


def layout_text(genome: np.ndarray, starts: np.ndarray, lengths: np.ndarray,
                err_rate: float, rng_err: np.random.Generator | None) -> np.ndarray:
    """Copy each read out of ``genome`` (codes), apply i.i.d. substitutions (each base with
    probability ``err_rate`` becomes one of the other three, uniformly), and write the ASCII
    text with a '$' after every read."""
    starts = np.asarray(starts, dtype=np.int64)
    lengths = np.asarray(lengths, dtype=np.int64)
    m = lengths.size
    total = int(lengths.sum()) + m
    text = np.empty(total, dtype=np.uint8)
    ends = np.cumsum(lengths + 1)            # one past each read's separator
    begins = ends - lengths - 1
    for c0 in range(0, m, _CHUNK_READS):
        c1 = min(m, c0 + _CHUNK_READS)
        lo, hi = int(begins[c0]), int(ends[c1 - 1])
        seg_len = hi - lo
        rel_begin = begins[c0:c1] - lo
        # genome index for every byte of the chunk (separator slots are overwritten below)
        gidx = np.repeat(starts[c0:c1] - rel_begin, lengths[c0:c1] + 1) + np.arange(seg_len)
        is_sep = np.zeros(seg_len, dtype=bool)
        is_sep[(ends[c0:c1] - 1) - lo] = True
        gidx[is_sep] = 0
        codes = genome[gidx]
        if err_rate > 0.0:
            hit = rng_err.random(seg_len) < err_rate
            hit &= ~is_sep
            k = int(hit.sum())
            codes[hit] = (codes[hit] + rng_err.integers(1, 4, size=k, dtype=np.uint8)) & 3
        chunk = _ASCII[codes]
        chunk[is_sep] = SEP
        text[lo:hi] = chunk
    return text


def text_from_strings(reads) -> np.ndarray:
    """Concatenate byte strings, each followed by '$' (used for hand-written cases)."""
    parts = []
    for r in reads:
        if isinstance(r, str):
            r = r.encode()
        parts.append(bytes(r) + b"$")
    return np.frombuffer(b"".join(parts), dtype=np.uint8).copy()


def _uniform_reads(index, name, g, m, read_len, err, min_len, genome=None):
    r_genome, r_starts, r_err = _rngs(index, 3)
    if genome is None:
        genome = random_genome(r_genome, g)
    starts = r_starts.integers(0, g - read_len + 1, size=m, dtype=np.int64)
    lengths = np.full(m, read_len, dtype=np.int64)
    text = layout_text(genome, starts, lengths, err, r_err)
    return ReadSet(name, text, starts, lengths, min_len, g,
                   dict(genome_len=g, reads=m, read_len=read_len, err=err))


def small_plain(index: int = 0) -> ReadSet:
    """20,000-base genome, 400 error-free reads of 200 bp (4x), overlaps >= 30."""
    return _uniform_reads(index, "plain-small-20k", 20_000, 400, 200, 0.0, 30)


def large_plain(index: int = 1, scale: float = 1.0) -> ReadSet:
    """5 Mbp genome, 100,000 reads of 500 bp (10x), 0.5 % substitutions, overlaps >= 40.

    ``scale`` < 1 shrinks genome and read count together (same coverage, read length and error
    rate): used for bounded CPU samples of the same workload."""
    g = int(round(5_000_000 * scale))
    m = int(round(100_000 * scale))
    name = "plain-large-5M" if scale == 1.0 else f"plain-large-5M-x{scale:g}"
    return _uniform_reads(index, name, g, m, 500, 0.005, 40)


def repeat_genome(rng: np.random.Generator, g: int = 40_000_000, n_copies: int = 50,
                  rep_len: int = 5000, rep_div: float = 0.01, n_tandem: int = 2000,
                  unit_lo: int = 2, unit_hi: int = 64, cp_lo: int = 10, cp_hi: int = 200) -> np.ndarray:
    """i.i.d. background with ``n_copies`` diverged copies of one random consensus and
    ``n_tandem`` tandem arrays, all written at non-overlapping uniform positions."""
    genome = random_genome(rng, g)
    consensus = random_genome(rng, rep_len)
    segs = []
    for _ in range(n_copies):
        c = consensus.copy()
        hit = rng.random(rep_len) < rep_div
        c[hit] = (c[hit] + rng.integers(1, 4, size=int(hit.sum()), dtype=np.uint8)) & 3
        segs.append(c)
    for _ in range(n_tandem):
        u = int(rng.integers(unit_lo, unit_hi + 1))
        k = int(rng.integers(cp_lo, cp_hi + 1))
        unit = random_genome(rng, u)
        segs.append(np.tile(unit, k))
    order = rng.permutation(len(segs))
    total = sum(s.size for s in segs)
    free = g - total
    assert free > 0
    cuts = np.sort(rng.integers(0, free + 1, size=len(segs)))
    pos = 0
    prev_cut = 0
    for slot, si in enumerate(order):
        pos += int(cuts[slot]) - prev_cut
        prev_cut = int(cuts[slot])
        s = segs[si]
        genome[pos:pos + s.size] = s
        pos += s.size
    return genome


def repeat_stress(index: int = 4, scale: float = 1.0) -> ReadSet:
    """40 Mbp repeat-rich genome, 400,000 reads of 1,000 bp (10x), 1 % substitutions,
    overlaps >= 100.  ``scale`` shrinks genome, repeat counts and reads together."""
    r_genome, r_starts, r_err = _rngs(index, 3)
    g = int(round(40_000_000 * scale))
    genome = repeat_genome(r_genome, g, n_copies=max(1, int(round(50 * scale))),
                           n_tandem=max(1, int(round(2000 * scale))))
    m = int(round(400_000 * scale))
    L = 1000
    starts = r_starts.integers(0, g - L + 1, size=m, dtype=np.int64)
    lengths = np.full(m, L, dtype=np.int64)
    text = layout_text(genome, starts, lengths, 0.01, r_err)
    name = "repeat-stress-40M" if scale == 1.0 else f"repeat-stress-40M-x{scale:g}"
    return ReadSet(name, text, starts, lengths, 100, g,
                   dict(genome_len=g, reads=m, read_len=L, err=0.01))


def _variable_set(rng_g, rng_s, rng_e, g, len_lo, len_hi, coverage, err, min_len, name):
    genome = random_genome(rng_g, g)
    hi = min(len_hi, g)
    lo = min(len_lo, hi)
    lengths = []
    total = 0
    target = coverage * g
    while total < target:
        L = int(rng_s.integers(lo, hi + 1))
        lengths.append(L)
        total += L
    lengths = np.asarray(lengths, dtype=np.int64)
    starts = (rng_s.random(lengths.size) * (g - lengths + 1)).astype(np.int64)
    text = layout_text(genome, starts, lengths, err, rng_e)
    return ReadSet(name, text, starts, lengths, min_len, g,
                   dict(genome_len=g, reads=int(lengths.size), coverage=coverage, err=err))


def batched_sets(index: int = 2, n_sets: int = 256, g_lo: int = 10_000, g_hi: int = 2_000_000,
                 max_total: int | None = None) -> list:
    """Independent fragment sets: genome length log-uniform [g_lo, g_hi], read lengths uniform
    100..1000, coverage uniform 5..20x, 0.5 % substitutions, overlaps >= 40."""
    (r_top,) = _rngs(index, 1)
    sets = []
    total = 0
    for s in range(n_sets):
        rg, rs, re = [np.random.Generator(np.random.PCG64(c))
                      for c in np.random.SeedSequence(SEED_BASE + index, spawn_key=(s,)).spawn(3)]
        g = int(round(math.exp(r_top.uniform(math.log(g_lo), math.log(g_hi)))))
        cov = float(r_top.uniform(5.0, 20.0))
        rset = _variable_set(rg, rs, re, g, 100, 1000, cov, 0.005, 40, f"set{s}")
        sets.append(rset)
        total += rset.n
        if max_total is not None and total >= max_total:
            break
    return sets


def serving_jobs(index: int = 3, n_jobs: int = 2000, rate_per_s: float = 1.0,
                 g_lo: int = 1_000, g_hi: int = 5_000_000):
    """Poisson stream of assembly jobs: genome length log-uniform [g_lo, g_hi], reads uniform
    150..min(800, G), 8x coverage, 0.5 % substitutions, overlaps >= 40.  Returns
    (arrival_times_s, [ReadSet, ...])."""
    arrivals, sizes = serving_plan(index, n_jobs, rate_per_s, g_lo, g_hi)
    return arrivals, [serving_job(index, j, g) for j, g in enumerate(sizes)]


def serving_plan(index: int = 3, n_jobs: int = 2000, rate_per_s: float = 1.0,
                 g_lo: int = 1_000, g_hi: int = 5_000_000):
    """Arrival times and genome lengths of the serving stream (the draws serving_jobs makes
    before generating each job's reads)."""
    (r_top,) = _rngs(index, 1)
    gaps = r_top.exponential(1.0 / rate_per_s, size=n_jobs)
    arrivals = np.cumsum(gaps) - gaps[0]
    sizes = [int(round(math.exp(r_top.uniform(math.log(g_lo), math.log(g_hi)))))
             for _ in range(n_jobs)]
    return arrivals, sizes


def serving_job(index: int, j: int, g: int) -> ReadSet:
    """Job j of the serving stream with genome length g: its reads depend only on (index, j,
    g), so jobs can be generated independently (and in parallel)."""
    rg, rs, re = [np.random.Generator(np.random.PCG64(c))
                  for c in np.random.SeedSequence(SEED_BASE + index, spawn_key=(j,)).spawn(3)]
    return _variable_set(rg, rs, re, g, 150, 800, 8.0, 0.005, 40, f"job{j}")


def random_dna_reads(seed: int, m: int, len_lo: int, len_hi: int, alphabet: bytes = b"ACGT",
                     allow_empty: bool = False) -> np.ndarray:
    """Independent random reads (no genome): lengths uniform [len_lo, len_hi] (0 allowed if
    ``allow_empty``), letters uniform over ``alphabet``.  For ragged parity cases."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, seed])))
    lo = len_lo if allow_empty else max(1, len_lo)
    lengths = rng.integers(lo, len_hi + 1, size=m)
    alpha = np.frombuffer(alphabet, dtype=np.uint8)
    parts = []
    for L in lengths:
        parts.append(alpha[rng.integers(0, alpha.size, size=int(L))])
        parts.append(np.array([SEP], dtype=np.uint8))
    return np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint8)


def genome_reads(seed: int, g: int, m: int, read_len: int, err: float = 0.0,
                 alphabet_size: int = 4) -> np.ndarray:
    """Small overlapping-read text: reads of ``read_len`` from one random genome over the first
    ``alphabet_size`` bases, with i.i.d. substitutions.  For parity cases with real overlaps."""
    rng_g, rng_s, rng_e = [np.random.Generator(np.random.PCG64(c))
                           for c in np.random.SeedSequence([SEED_BASE, 7, seed]).spawn(3)]
    genome = rng_g.integers(0, alphabet_size, size=g, dtype=np.uint8)
    starts = rng_s.integers(0, g - read_len + 1, size=m, dtype=np.int64)
    lengths = np.full(m, read_len, dtype=np.int64)
    return layout_text(genome, starts, lengths, err, rng_e)


WORKLOADS = {
    "plain-small-20k": small_plain,
    "plain-large-5M": large_plain,
    "repeat-stress-40M": repeat_stress,
}


def lookup_patterns(text: np.ndarray, count: int, seed: int, len_lo: int = 0,
                    len_hi: int = 80) -> list:
    """Seeded query strings for pattern lookup on ``text``: half are substrings of the text
    (cut before the first separator they would cross), a quarter are read prefixes and a
    quarter are uniform random A/C/G/T strings (mostly absent).  Lengths uniform in
    [len_lo, len_hi]."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, 11, seed])))
    tb = bytes(np.asarray(text, dtype=np.uint8))
    starts = [0] + [i + 1 for i, c in enumerate(tb[:-1]) if c == ord("$")]
    out = []
    for j in range(count):
        L = int(rng.integers(len_lo, len_hi + 1))
        kind = j % 4
        if kind in (0, 1):
            p = int(rng.integers(0, len(tb)))
        elif kind == 2:
            p = starts[int(rng.integers(0, len(starts)))]
        else:
            out.append(bytes(rng.choice(list(b"ACGT"), size=L).astype(np.uint8)))
            continue
        s = tb[p:p + L]
        cut = s.find(b"$")
        out.append(s if cut < 0 else s[:cut])
    return out


def two_cuttings(seed: int, length: int, mean_frag: int, alphabet: bytes = b"ACGT",
                 min_gap: int = 1):
    """A random sequence cut twice at disjoint sets of interior positions (the setting of the
    cut-and-continue reconstruction): returns (text of the shuffled fragments joined with '$',
    the sequence, the fragments in text order).  Each cutting has about length/mean_frag
    pieces; no interior cut position is shared, and all cut positions of both cuttings lie on
    multiples of ``min_gap`` (so every fragment has at least that many bases)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, 13, seed])))
    seq = bytes(rng.choice(list(alphabet), size=length).astype(np.uint8))
    k = max(1, length // mean_frag - 1)
    slots = np.arange(1, (length - 1) // min_gap + 1) * min_gap
    pos = rng.choice(slots, size=min(2 * k, slots.size), replace=False)
    a, b = np.sort(pos[: len(pos) // 2]), np.sort(pos[len(pos) // 2:])
    frags = []
    for cuts in (a, b):
        edges = [0] + [int(c) for c in cuts] + [length]
        frags += [seq[x:y] for x, y in zip(edges, edges[1:])]
    perm = rng.permutation(len(frags))
    frags = [frags[i] for i in perm]
    return text_from_strings([f.decode() for f in frags]), seq, frags


def strand_reads(seed: int, g: int, m: int, read_len: int):
    """Error-free reads of one random genome taken from either strand: returns (text, starts,
    strands) with strand 1 meaning the read is the reverse complement of
    genome[start:start+read_len].  For ground-truth checks of overlaps on both strands."""
    rng_g, rng_s = [np.random.Generator(np.random.PCG64(c))
                    for c in np.random.SeedSequence([SEED_BASE, 17, seed]).spawn(2)]
    genome = rng_g.integers(0, 4, size=g, dtype=np.uint8)
    starts = rng_s.integers(0, g - read_len + 1, size=m)
    strands = rng_s.integers(0, 2, size=m)
    letters = np.frombuffer(b"ACGT", dtype=np.uint8)
    reads = []
    for s, d in zip(starts.tolist(), strands.tolist()):
        codes = genome[s:s + read_len]
        if d:
            codes = 3 - codes[::-1]  # A<->T, C<->G under the code order A C G T
        reads.append(bytes(letters[codes]))
    return text_from_strings(reads), starts, strands
