"""Cut-and-continue reconstruction from the fragments of two cuttings, on plain strings.

TEST INFRASTRUCTURE ONLY (see the package header).  This follows the procedure of Sec. III
step by step with direct prefix tests (``bytes.startswith``) instead of suffix-array searches:

* A 'fir' pair is two fragments one of which is a proper prefix of the other; it holds the first
  fragment of each cutting (two equal fragments only when they are all there is).  Pairs are tried with the longer fragment b in increasing id, then
  the shorter a in increasing id.
* State: the sequence so far RS and the lengths e_lo <= e_hi that the two cuttings cover.  The
  remainder r = RS[e_lo:e_hi] is the uncovered end of the cutting that is ahead; the cutting that
  is behind takes the next fragment f, which must start with r (|f| > |r|: RS grows by
  f[|r|:] and the cuttings swap roles) or be a proper prefix of r (|f| < |r|: the remainder
  shrinks).  |f| == |r| only for the last fragment, when both cuttings end together.
* Candidates are tried in increasing id; a dead end returns to the last choice (back-tracking).
  The first complete reconstruction -- every fragment placed, both cuttings ending at |RS| -- is
  returned as (RS, placement order), or None.
"""
from __future__ import annotations


def _candidates(frags, used, r, last):
    out = []
    for f, s in enumerate(frags):
        if used[f]:
            continue
        if len(s) > len(r) and s.startswith(r):
            out.append(f)
        elif len(s) < len(r) and r.startswith(s):
            out.append(f)
        elif len(s) == len(r) and last and s == r:
            out.append(f)
    return out


def fir_pairs(frags):
    """(b, a): a is a proper prefix of b; with exactly two fragments also an equal pair (both
    cuttings are the uncut sequence)."""
    m = len(frags)
    return [(b, a) for b in range(m) for a in range(m)
            if a != b and frags[b].startswith(frags[a])
            and (len(frags[a]) < len(frags[b]) or m == 2)]


def reconstruct(frags, max_steps=10 ** 7):
    frags = [bytes(f) for f in frags]
    m = len(frags)
    steps = 0
    for b, a in fir_pairs(frags):
        used = [False] * m
        used[a] = used[b] = True
        order = [a, b]
        rs = frags[b]
        e_lo, e_hi = len(frags[a]), len(frags[b])
        if m == 2 and e_lo == e_hi:
            return rs, order
        # explicit stack of (saved state, candidates, next index)
        def frame():
            r = rs[e_lo:e_hi]
            cand = _candidates(frags, used, r, len(order) == m - 1) if e_lo < e_hi else []
            return [(rs, e_lo, e_hi, len(order)), cand, 0]
        stack = [frame()]
        while stack:
            steps += 1
            if steps > max_steps:
                return None
            top = stack[-1]
            rs, e_lo, e_hi, k = top[0]
            for f in order[k:]:
                used[f] = False
            del order[k:]
            if top[2] >= len(top[1]):
                stack.pop()
                continue
            f = top[1][top[2]]
            top[2] += 1
            s = frags[f]
            used[f] = True
            order.append(f)
            rlen = e_hi - e_lo
            if len(s) > rlen:
                rs = rs + s[rlen:]
                e_lo, e_hi = e_hi, e_lo + len(s)
            else:
                e_lo = e_lo + len(s)
            if len(order) == m and e_lo == e_hi:
                return rs, list(order)
            stack.append(frame())
    return None
