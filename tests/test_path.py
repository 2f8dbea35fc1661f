"""The weighted overlap graph's maximal Hamiltonian path (Sec. III).

Oracle pins (oracle/path.py, CPU): the paper's worked example -- its printed path is the unique
maximum (15) over all 120 orders and merges to its printed superstring -- closed forms, and a
planted mistake.  The library's host search (sa_overlap_path through the C ABI, CPU only: it is
host code) against the oracle: the worked example, random weighted graphs (the exact search's
weight equals the exhaustive maximum; its order is a valid path of that weight), the greedy rule
step for step, and argument checks.  The GPU-built overlaps feed the same search in
tests/test_gpu_parity.py."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import path as opath
from paper_1404_3456_amd import _abi, synth
from tests.test_oracle import _golden


def worked():
    frags, printed, superstring = _golden()
    frags = [f.encode() for f in frags]
    text = synth.text_from_strings(frags)
    rows = oracle.overlaps(text, 1)
    order = [frags.index(p.encode()) for p in printed]
    return frags, text, rows, order, superstring.encode()


# ---- oracle pins ---------------------------------------------------------------------------

def test_oracle_worked_example():
    frags, _, rows, order, superstring = worked()
    w = opath.weights(rows)
    assert opath.best_weight_exhaustive(5, w) == 15 == opath.path_weight(order, w)
    at_best = [o for o in itertools.permutations(range(5)) if opath.path_weight(o, w) == 15]
    assert at_best == [tuple(order)]
    assert opath.merge(frags, order, w) == superstring
    assert len(superstring) == 28


def test_oracle_closed_forms():
    # every pair overlapping by the same length: any order weighs (m - 1) * l
    m, ell = 6, 3
    w = {(a, b): ell for a in range(m) for b in range(m) if a != b}
    assert opath.best_weight_exhaustive(m, w) == (m - 1) * ell
    # a chain cut from one string with overlaps 5, 4, 3: the chain is the only maximum, and the
    # greedy rule finds it too
    s = b"ACGTACCGTTAGGCATTACGA"
    frags = [s[0:9], s[4:13], s[9:17], s[14:21]]
    text = synth.text_from_strings(frags)
    w = opath.weights(oracle.overlaps_brute(text, 1))
    assert opath.best_weight_exhaustive(4, w) == opath.path_weight([0, 1, 2, 3], w) == 5 + 4 + 3
    assert opath.greedy_path(4, w) == [0, 1, 2, 3]
    assert opath.merge(frags, [0, 1, 2, 3], w) == s
    # no edges: the fragments laid end to end in id order
    assert opath.greedy_path(3, {}) == [0, 1, 2]


def test_oracle_planted_merge_mistake_is_caught():
    frags, _, rows, order, superstring = worked()
    w = opath.weights(rows)
    shorter = {k: v - 1 for k, v in w.items()}  # merging past one base too few
    assert opath.merge(frags, order, shorter) != superstring


# ---- the library's host search against the oracle ------------------------------------------

def test_library_worked_example():
    frags, text, rows, order, superstring = worked()
    got_order, weight, rs = _abi.sa_overlap_path(text, rows)
    assert got_order == order and weight == 15 and rs == superstring


def _random_graph(rng, m, flen=40):
    frags = [bytes(rng.choice(list(b"ACGT"), size=flen).tolist()) for _ in range(m)]
    text = synth.text_from_strings(frags)
    rows = []
    for a in range(m):
        for b in range(m):
            if a != b and rng.random() < 0.5:
                rows.append((a, b, int(rng.integers(1, flen + 1))))
    return frags, text, np.array(rows, dtype=np.int32).reshape(-1, 3)


@pytest.mark.parametrize("seed", range(12))
def test_library_exact_matches_exhaustive(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 9))
    frags, text, rows = _random_graph(rng, m)
    w = opath.weights(rows)
    order, weight, rs = _abi.sa_overlap_path(text, rows, exact_max_m=16)
    assert sorted(order) == list(range(m))
    assert weight == opath.path_weight(order, w) == opath.best_weight_exhaustive(m, w)
    assert rs == opath.merge(frags, order, w)


@pytest.mark.parametrize("seed", range(6))
def test_library_greedy_matches_oracle_rule(seed):
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(10, 60))
    frags, text, rows = _random_graph(rng, m)
    w = opath.weights(rows)
    order, weight, rs = _abi.sa_overlap_path(text, rows, exact_max_m=0)
    assert order == opath.greedy_path(m, w)
    assert weight == opath.path_weight(order, w)
    assert rs == opath.merge(frags, order, w)


def test_library_exact_up_to_twenty_fragments():
    rng = np.random.default_rng(7)
    frags, text, rows = _random_graph(rng, 14, flen=30)
    w = opath.weights(rows)
    order, weight, _ = _abi.sa_overlap_path(text, rows, exact_max_m=20)
    g_order, g_weight, _ = _abi.sa_overlap_path(text, rows, exact_max_m=0)
    assert sorted(order) == list(range(14)) and weight == opath.path_weight(order, w)
    assert weight >= g_weight  # the exact search is never below the greedy rule


def test_library_argument_checks():
    text = synth.text_from_strings([b"ACGT", b"CGTA"])
    for bad in ([(0, 0, 1)], [(0, 2, 1)], [(0, 1, 5)], [(-1, 1, 1)]):
        with pytest.raises(_abi.SaasmError) as e:
            _abi.sa_overlap_path(text, np.array(bad, dtype=np.int32))
        assert e.value.code == _abi.SA_ERR_INVALID
    with pytest.raises(_abi.SaasmError):
        _abi.sa_overlap_path(text, np.zeros((0, 3), dtype=np.int32), exact_max_m=21)
    assert _abi.sa_overlap_path(text, np.array([(0, 1, 3)], dtype=np.int32)) == ([0, 1], 3, b"ACGTA")
