"""The skew (difference-cover-3) recursion read for a text with many separators, checked on the
CPU against the suffix-array definition.

The GPU construction relies on these choices, which the cited linear-work construction (it
assumes a single sentinel) does not spell out for many distinct separators:
  * top-level symbols are 0 for a separator and 1..4 for A, C, G, T, and two symbols 0 compare
    by position (separator r below separator r+1);
  * a sample triple that holds a separator has its symbols after the separator set to 0 and
    gets a name of its own, in position order;
  * no dummy sample is added when a level's length is 1 mod 3, because the last symbol of every
    level is unique;
  * suffixes at positions 0 mod 3 that start with a separator sort by position.
This module restates the recursion with those choices in plain Python (slow; small texts only)
and compares it with brute force on every short text and on random and repetitive ones.  It
shares nothing with the GPU code or with the oracle.
"""
import itertools
import random

SYM = {"$": 0, "A": 1, "C": 2, "G": 3, "T": 4}


def brute_sa(text):
    """The definition: sort suffixes over the alphabet $_0 < $_1 < ... < A < C < G < T."""
    m = text.count("$")
    ints, r = [], 0
    for ch in text:
        if ch == "$":
            ints.append(r)
            r += 1
        else:
            ints.append(m + SYM[ch])
    return sorted(range(len(text)), key=lambda p: ints[p:])


def skew(n, sym, top, own_names=True):
    """Suffix array of a level of n symbols; sym(p) gives symbol p (0 past the end).
    own_names=False names separator triples by content alone (a planted mistake)."""
    n0, n1 = (n + 2) // 3, (n + 1) // 3
    n12 = n - n0
    rank = {n: 0, n + 1: 0, n + 2: 0}
    sa12 = []
    if n12:
        samples = [3 * (j >> 1) + 1 + (j & 1) for j in range(n12)]
        if top:
            def key(p):
                c0 = sym(p)
                c1 = sym(p + 1) if c0 and p + 1 < n else 0
                c2 = sym(p + 2) if c1 and p + 2 < n else 0
                return (c0, c1, c2)
            order = sorted(samples, key=key)  # stable: equal keys stay in position order
            heads = [j == 0 or key(order[j]) != key(order[j - 1])
                     or (own_names and key(order[j])[2] == 0) for j in range(n12)]
        else:
            def key(p):
                return (sym(p), sym(p + 1), sym(p + 2))
            order = sorted(samples, key=key)
            heads = [j == 0 or key(order[j]) != key(order[j - 1]) for j in range(n12)]
        names, name = [0] * (n12 + 3), 0
        for j, p in enumerate(order):
            name += heads[j]
            names[p // 3 if p % 3 == 1 else n1 + p // 3] = name
            rank[p] = name
        sa12 = order
        if name < n12:  # names repeat: rank the samples by the name string's suffix array
            sub = skew(n12, lambda q: names[q], False)
            sa12 = [3 * r + 1 if r < n1 else 3 * (r - n1) + 2 for r in sub]
            for k, p in enumerate(sa12):
                rank[p] = k + 1

    def key0(i):  # (symbol, rank of the next suffix); separators by position
        c = sym(i)
        return (c, i if c == 0 else rank[i + 1])
    rest = sorted(range(0, n, 3), key=key0)

    def before(a, b):  # a = 0 mod 3, b a sample
        if sym(a) != sym(b):
            return sym(a) < sym(b)
        if sym(a) == 0:
            return a < b
        if b % 3 == 1:
            return rank[a + 1] < rank[b + 1]
        if sym(a + 1) != sym(b + 1):
            return sym(a + 1) < sym(b + 1)
        if sym(a + 1) == 0:
            return a < b
        return rank[a + 2] < rank[b + 2]

    out, i, j = [], 0, 0
    while i < len(rest) or j < len(sa12):
        if j == len(sa12) or (i < len(rest) and before(rest[i], sa12[j])):
            out.append(rest[i])
            i += 1
        else:
            out.append(sa12[j])
            j += 1
    return out


def skew_sa(text, own_names=True):
    n = len(text)
    return skew(n, lambda p: SYM[text[p]] if p < n else 0, True, own_names)


def test_every_short_text():
    """All texts over {$, A, C} of length <= 8 that end with '$' (3,280 texts)."""
    count = 0
    for L in range(1, 9):
        for body in itertools.product("$AC", repeat=L - 1):
            t = "".join(body) + "$"
            assert skew_sa(t) == brute_sa(t), t
            count += 1
    assert count == sum(3 ** k for k in range(8))


def test_every_length_mod_three_and_deep_recursion():
    for k in range(1, 200):
        for t in ("A" * k + "$", "AC" * k + "$", "A" * k + "$" + "A" * (k // 2) + "$"):
            assert skew_sa(t) == brute_sa(t), t


def test_random_and_repetitive_read_sets():
    rng = random.Random(1404)
    for _ in range(1500):
        reads = []
        for _ in range(rng.randint(1, 6)):
            L = rng.choice([0, 0, 1, 2, 3, 5, 8, 13, 30])
            alpha = rng.choice(["A", "AC", "ACGT"])
            reads.append("".join(rng.choice(alpha) for _ in range(L)))
        if rng.random() < 0.3:
            reads += reads[: rng.randint(1, len(reads))]
        t = "$".join(reads) + "$"
        assert skew_sa(t) == brute_sa(t), t


def test_planted_mistake_content_names():
    """Naming a triple that holds a separator by its content alone (enough with a single
    sentinel) gives wrong arrays once there are several separators, so the checks above are
    not vacuous."""
    wrong = []
    for L in range(1, 8):
        for body in itertools.product("$AC", repeat=L - 1):
            t = "".join(body) + "$"
            if skew_sa(t, own_names=False) != brute_sa(t):
                wrong.append(t)
    assert wrong, "the separator naming rule made no difference"
