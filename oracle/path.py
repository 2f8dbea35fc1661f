"""Reading a reconstruction off the weighted overlap graph (Sec. III) -- TEST INFRASTRUCTURE ONLY.

Only the test suite calls this module; the GPU library neither imports nor runs it, and it
imports nothing from the library.

The graph has one vertex per fragment and an edge a -> b weighted by l(a, b), the longest
suffix-prefix overlap of a and b (the overlap rows; a pair with no row weighs 0).  The paper
takes a Hamiltonian path of maximal total weight through it and merges the fragments along the
path: each next fragment contributes what lies beyond its overlap with the one before.

* ``best_weight_exhaustive``: the definition itself -- every order of the fragments -- for a
  handful of fragments only.
* ``greedy_path``: the stated rule used above the exact search's size, taken step by step:
  edges by weight (heaviest first, then by a, then by b); an edge is kept when a has no
  successor yet, b no predecessor, and a and b are not already in one chain; the chains that
  remain are laid end to end in order of their first fragment.
* ``merge``: the superstring along an order.
"""
from __future__ import annotations

import itertools


def weights(rows):
    """{(a, b): l} from overlap rows."""
    return {(int(a), int(b)): int(l) for a, b, l in rows}


def path_weight(order, w):
    return sum(w.get((x, y), 0) for x, y in zip(order, order[1:]))


def best_weight_exhaustive(m, w):
    """Largest total weight of any order of m fragments (m <= 9)."""
    if m > 9:
        raise ValueError("exhaustive search is for a handful of fragments")
    if m == 0:
        return 0
    return max(path_weight(o, w) for o in itertools.permutations(range(m)))


def greedy_path(m, w):
    succ = [None] * m
    pred = [None] * m
    chain = list(range(m))  # chain id of each fragment (the id of its chain's first fragment)
    for (a, b), l in sorted(w.items(), key=lambda e: (-e[1], e[0][0], e[0][1])):
        if a == b or succ[a] is not None or pred[b] is not None or chain[a] == chain[b]:
            continue
        succ[a], pred[b] = b, a
        old, new = chain[b], chain[a]
        chain = [new if c == old else c for c in chain]
    order = []
    for h in range(m):
        if pred[h] is None:
            x = h
            while x is not None:
                order.append(x)
                x = succ[x]
    return order


def merge(frags, order, w):
    """Superstring along `order`: the first fragment, then each next one past its overlap."""
    if not order:
        return b""
    out = bytes(frags[order[0]])
    for x, y in zip(order, order[1:]):
        out += bytes(frags[y][w.get((x, y), 0):])
    return out
