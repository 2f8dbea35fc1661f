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
