"""Pins of the cut-and-continue reconstruction oracle (oracle/recon.py).  CPU only."""
import itertools
import os
import random

import pytest

from oracle import recon
from paper_1404_3456_amd import synth


def valid_two_cuttings(frags):
    """Brute force: every sequence X such that the fragments split into two groups, each of
    which tiles X in some order, with no interior cut position shared by the two groups."""
    m = len(frags)
    out = set()
    for perm in itertools.permutations(range(m)):
        for k in range(1, m):
            ga, gb = perm[:k], perm[k:]
            x = b"".join(frags[i] for i in ga)
            if x != b"".join(frags[i] for i in gb):
                continue
            cuts = lambda g: set(itertools.accumulate(len(frags[i]) for i in g[:-1]))
            if cuts(ga) & cuts(gb):
                continue
            out.add(x)
    return out


def is_valid(frags, rs, order):
    """The placement order uses every fragment once and splits into two cuttings that both tile
    rs (each fragment goes to the cutting that is behind) with no interior cut in common."""
    e = [0, 0]
    cuts = [set(), set()]
    for f in order:
        c = 0 if e[0] <= e[1] else 1
        s = frags[f]
        if rs[e[c]:e[c] + len(s)] != s:
            return False
        e[c] += len(s)
        cuts[c].add(e[c])
    interior = (cuts[0] & cuts[1]) - {len(rs)}
    return sorted(order) == list(range(len(frags))) and e[0] == e[1] == len(rs) and not interior


def tiny_instances(count, seed):
    rng = random.Random(seed)
    out = []
    for _ in range(count):
        L = rng.randint(3, 9)
        s = bytes(rng.choice(b"AC") for _ in range(L))
        pos = list(range(1, L))
        rng.shuffle(pos)
        ka, kb = rng.randint(0, 2), rng.randint(0, 2)
        a, b = sorted(pos[:ka]), sorted(pos[ka:ka + kb])
        frags = []
        for cuts in (a, b):
            edges = [0] + cuts + [L]
            frags += [s[x:y] for x, y in zip(edges, edges[1:])]
        rng.shuffle(frags)
        if rng.random() < 0.2:  # sometimes corrupt one fragment: may become unsolvable
            i = rng.randrange(len(frags))
            frags[i] = frags[i][:-1] + (b"C" if frags[i][-1:] == b"A" else b"A")
        out.append(frags)
    return out


TINY = tiny_instances(400, 1)


def test_tiny_vs_brute_force():
    """Back-tracking is complete: a reconstruction is returned exactly when one exists, and it
    is one of the valid ones."""
    solvable = 0
    for frags in TINY:
        want = valid_two_cuttings(frags)
        got = recon.reconstruct(frags)
        if want:
            solvable += 1
            assert got is not None, frags
            assert got[0] in want and is_valid(frags, *got), frags
        else:
            assert got is None, frags
    assert 100 < solvable < len(TINY)


@pytest.mark.parametrize("seed", range(4))
def test_random_cuttings_ground_truth(seed):
    """Random sequences cut at positions at least 16 apart: the reconstruction is the original
    sequence (shorter pieces can admit several answers, all valid)."""
    _, seq, frags = synth.two_cuttings(seed, 2000, 60, min_gap=16)
    rs, order = recon.reconstruct(frags)
    assert rs == seq and is_valid(frags, rs, order)


def test_backtracking_needed():
    """Sec. III: a short first fragment that is a prefix of two others.  Taking the wrong one
    first leads to a dead end; the search must go back and take the other."""
    # sequence ACACGT; cutting A: AC | ACGT, cutting B: ACA | CGT.  'AC' is a prefix of both
    # 'ACGT' and 'ACA'; the first pair tried (ACGT, AC) leaves the remainder GT, which no
    # fragment continues, so the search must go back and take (ACA, AC).
    frags = [b"AC", b"ACGT", b"ACA", b"CGT"]
    assert recon.fir_pairs(frags) == [(1, 0), (2, 0)]
    rs, order = recon.reconstruct(frags)
    assert rs == b"ACACGT" and order == [0, 2, 1, 3]
    # a case where the first 'fir' pair in search order is wrong
    seen_backtrack = False
    for frags in TINY:
        got = recon.reconstruct(frags)
        if got is None:
            continue
        first = recon.fir_pairs(frags)[0]
        if sorted(got[1][:2]) != sorted(first):
            seen_backtrack = True
            break
    assert seen_backtrack


def test_unsolvable():
    assert recon.reconstruct([b"AC", b"GT", b"TT"]) is None
    assert recon.reconstruct([b"ACGT", b"ACGA"]) is None
    assert recon.reconstruct([b"ACGT", b"ACGT"])[0] == b"ACGT"  # both cuttings left uncut
    assert recon.reconstruct([b"AC", b"AC", b"GT", b"GT"]) is None  # every cut would be shared


RECON_MUTANTS = {
    # no back-tracking: give up at the first dead end
    "no_backtrack": ("                stack.pop()\n                continue", "                return None"),
    # the sequence grows by the whole fragment instead of its part past the remainder
    "append_whole": ("rs = rs + s[rlen:]", "rs = rs + s"),
    # shorter candidates tested the wrong way round (remainder a prefix of the fragment)
    "prefix_reversed": ("elif len(s) < len(r) and r.startswith(s):", "elif len(s) < len(r) and s.startswith(r):"),
}


@pytest.mark.parametrize("name", sorted(RECON_MUTANTS))
def test_recon_planted_mistake_is_caught(name, tmp_path):
    src = open(recon.__file__).read()
    pat, rep = RECON_MUTANTS[name]
    assert pat in src
    p = tmp_path / "recon_mut.py"
    p.write_text(src.replace(pat, rep))
    ns = {}
    exec(compile(p.read_text(), str(p), "exec"), ns)
    caught = False
    for frags in TINY:
        want = valid_two_cuttings(frags)
        got = ns["reconstruct"](frags)
        if bool(want) != (got is not None) or (got is not None and (got[0] not in want or not is_valid(frags, *got))):
            caught = True
            break
    assert caught, name
