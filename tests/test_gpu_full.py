"""Parity at full workload sizes, in the launch configuration the benchmark times: outputs the
oracle can check at any size (permutation, sampled adjacent order and LCP, the Kasai property)
and the complete overlap set from the oracle's exact seed-and-verify search."""
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


def full_check(pkg, r, samples=400_000):
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
    rng = np.random.default_rng(r.n)
    idx = np.unique(np.concatenate([rng.integers(1, r.n, size=samples), [1, r.n - 1]]))
    bad, first = oracle.check_adjacent(r.text, sa, lcp, idx)
    assert bad == 0, f"first bad adjacent pair at {first}"
    assert lcp[0] == 0
    checks.assert_kasai_property(r.text, sa, lcp)
    want = oracle.overlaps(r.text, r.min_len)
    assert np.array_equal(ovl, want)
    return want.shape[0]


def test_full_plain_large(pkg):
    rows = full_check(pkg, synth.large_plain())
    assert rows > 100_000


def test_full_repeat_stress(pkg):
    rows = full_check(pkg, synth.repeat_stress(), samples=200_000)
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
    overlaps through the C ABI.  SA and LCP: permutation, the oracle's sampled adjacent order
    and LCP.  Overlaps: the exact positional truth of error-free reads from a random genome,
    and direct string checks of sampled rows."""
    text, starts, lengths = max_size_text()
    n = text.size
    print(f"max-size case: n={n}", flush=True)
    t = torch.from_numpy(text).cuda()
    sa, isa = pkg.sa_build(t)
    lcp = pkg.sa_lcp(t, sa, isa)
    ovl = pkg.sa_overlaps(t, sa, isa, lcp, 100)
    torch.cuda.synchronize()
    print("max-size case: GPU done", flush=True)
    sa, isa, lcp, ovl = sa.cpu().numpy(), isa.cpu().numpy(), lcp.cpu().numpy(), ovl.cpu().numpy()
    del t
    checks.assert_sa_basic(text, sa)
    assert np.array_equal(isa[sa], np.arange(n, dtype=np.int32))
    del isa
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([rng.integers(1, n, size=200_000), [1, n - 1]]))
    bad, first = oracle.check_adjacent(text, sa, lcp, idx)
    assert bad == 0, f"first bad adjacent pair at {first}"
    assert lcp[0] == 0
    del sa, lcp
    want = checks.positional_overlaps_ragged(starts, lengths, 100)
    assert np.array_equal(ovl, want)
    rows = ovl[np.sort(rng.choice(ovl.shape[0], size=2000, replace=False))]
    checks.assert_overlaps_valid(text, rows, 100)
    print(f"max-size case: {want.shape[0]} overlap rows checked", flush=True)
