"""Host search of sa_reconstruct (C ABI) against the string oracle, with the suffix array, its
inverse and the LCP array taken from the CPU oracle.  CPU only: the library's search is host
code; the GPU-built arrays are exercised in the GPU parity tests."""
import numpy as np
import pytest

import oracle
from oracle import recon
from paper_1404_3456_amd import _abi, synth
from tests.test_recon_oracle import TINY


def host_arrays(text):
    sa = oracle.suffix_array(text)
    isa = np.empty_like(sa)
    isa[sa] = np.arange(sa.size, dtype=np.int32)
    return sa, isa, oracle.lcp_array(text, sa)


def run(frags):
    text = synth.text_from_strings(frags)
    return _abi.sa_reconstruct_host(text, *host_arrays(text))


def test_tiny_matches_oracle():
    for frags in TINY:
        if any(len(f) == 0 for f in frags):
            continue
        want = recon.reconstruct(frags)
        got = run(frags)
        assert (got is None) == (want is None), frags
        if want is not None:
            assert got[0] == want[0] and got[1] == want[1], frags


@pytest.mark.parametrize("seed", range(3))
def test_random_cuttings(seed):
    _, seq, frags = synth.two_cuttings(seed, 3000, 50)
    got = run(frags)
    assert got == recon.reconstruct(frags)  # short fragments: several answers, same choice
    _, seq, frags = synth.two_cuttings(seed, 3000, 50, min_gap=16)
    got = run(frags)
    assert got == recon.reconstruct(frags) and got[0] == seq


def test_backtracking_example():
    got = run([b"AC", b"ACGT", b"ACA", b"CGT"])
    assert got == (b"ACACGT", [0, 2, 1, 3])


def test_rejects_bad_input():
    text = synth.text_from_strings([b"AC", b"ACG"])
    sa, isa, lcp = host_arrays(text)
    bad = sa.copy()
    bad[[0, 1]] = bad[[1, 0]]
    with pytest.raises(_abi.SaasmError):
        _abi.sa_reconstruct_host(text, bad, isa, lcp)
    t2 = synth.text_from_strings([b"AC", b"", b"ACG"])
    with pytest.raises(_abi.SaasmError):
        _abi.sa_reconstruct_host(t2, *host_arrays(t2))
