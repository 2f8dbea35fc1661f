"""The LCP entry point without allocation (sa_lcp_noalloc) against sa_lcp: identical arrays on
two calls in a row, the second with a smaller text, so the scratch the first call left behind
is reused; the size limit and a bad byte are reported as errors."""
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


def _arrays(pkg, text):
    t = torch.from_numpy(text).cuda()
    sa, isa = pkg.sa_build(t)
    return t, sa, isa


def test_noalloc_lcp_matches_sa_lcp_twice(pkg):
    big = synth.genome_reads(4401, 400_000, 12_000, 300, err=0.005)   # ~3.6 M characters
    small = synth.genome_reads(4402, 20_000, 700, 150, err=0.01)       # ~106 k characters
    assert big.size <= pkg.sa_lcp_noalloc_max_n()
    for text in (big, small):
        t, sa, isa = _arrays(pkg, text)
        want = pkg.sa_lcp(t, sa, isa, check=True)
        got = torch.full_like(want, -7)
        pkg.sa_lcp_noalloc(t, sa, isa, got, check=True)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
    # the second, smaller text also against the oracle
    w = oracle.lcp_array(small, oracle.suffix_array(small))
    assert np.array_equal(got.cpu().numpy(), w)


def test_noalloc_lcp_limits(pkg):
    lib = pkg.load()
    import ctypes
    n_max = pkg.sa_lcp_noalloc_max_n()
    one = torch.zeros(4, dtype=torch.int32, device="cuda")
    text = torch.zeros(4, dtype=torch.uint8, device="cuda")
    P = ctypes.c_void_p
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.sa_lcp_noalloc(P(text.data_ptr()), n_max + 1, P(one.data_ptr()), P(one.data_ptr()),
                            P(one.data_ptr()), s)
    assert rc == pkg.SA_ERR_TOO_LARGE
    assert b"2^24" in lib.sa_last_error()
    rc = lib.sa_lcp_noalloc(None, 4, P(one.data_ptr()), P(one.data_ptr()), P(one.data_ptr()), s)
    assert rc == pkg.SA_ERR_INVALID
    # a byte outside A, C, G, T, $ is found on the device and reported through lcp[0]
    bad = np.frombuffer(b"ACGTACGTA$CCGTN$", dtype=np.uint8).copy()
    ok = bad.copy()
    ok[14] = ord("A")
    t_ok, sa, isa = _arrays(pkg, ok)
    lcp = torch.zeros(ok.size, dtype=torch.int32, device="cuda")
    t_bad = torch.from_numpy(bad).cuda()
    with pytest.raises(pkg.SaasmError) as e:
        pkg.sa_lcp_noalloc(t_bad, sa, isa, lcp, check=True)
    assert e.value.code == pkg.SA_ERR_ALPHABET
