"""Pure-Python literal definitions, for tiny inputs only (test infrastructure).

These share no reasoning with ``saoracle.c``: instead of a byte comparator with a separator
rule, the text is mapped to integers -- the separator closing read i becomes the integer i, any
other byte v becomes m + v -- and suffixes are compared as Python lists.  That is the ordered
alphabet of the text written out (Sec. III fragments, Sec. IV suffix array), with no special
cases left to get wrong.
"""
from __future__ import annotations


def to_ints(text: bytes):
    m = text.count(b"$")
    out = []
    r = 0
    for v in text:
        if v == ord("$"):
            out.append(r)
            r += 1
        else:
            out.append(m + v)
    return out


def suffix_array(text: bytes):
    s = to_ints(text)
    return sorted(range(len(s)), key=lambda p: s[p:])


def lcp_array(text: bytes, sa):
    s = to_ints(text)
    out = [0] * len(sa)
    for i in range(1, len(sa)):
        p, q = sa[i - 1], sa[i]
        k = 0
        while p + k < len(s) and q + k < len(s) and s[p + k] == s[q + k]:
            k += 1
        out[i] = k
    return out


def reads(text: bytes):
    return text.split(b"$")[:-1]


def overlaps(text: bytes, min_len: int):
    rs = reads(text)
    out = []
    for a, ra in enumerate(rs):
        for b, rb in enumerate(rs):
            if a == b:
                continue
            best = 0
            for l in range(min_len, min(len(ra), len(rb)) + 1):
                if ra[len(ra) - l:] == rb[:l]:
                    best = l
            if best:
                out.append((a, b, best))
    return out


def lookup(text: bytes, pattern: bytes):
    """[lo, hi): the positions of the literal suffix array whose suffixes start with pattern
    (the pattern's bytes mapped like the text's non-separator bytes)."""
    s = to_ints(text)
    m = text.count(b"$")
    pat = [m + v for v in pattern]
    hits = [i for i, p in enumerate(suffix_array(text)) if s[p:p + len(pat)] == pat]
    if not hits:  # empty interval: its place is the number of smaller suffixes
        lo = sum(1 for p in range(len(s)) if s[p:] < pat)
        return lo, lo
    return hits[0], hits[-1] + 1


_COMP = {ord("A"): ord("T"), ord("C"): ord("G"), ord("G"): ord("C"), ord("T"): ord("A")}


def revcomp(read: bytes) -> bytes:
    return bytes(_COMP.get(c, c) for c in reversed(read))


def overlaps_rc(text: bytes, min_len: int):
    """Both strands, literally: for reads a != b and each of the three ways two reads can
    meet -- (A, B) = (a, b) [strand 0], (a, revcomp(b)) [1], (revcomp(a), b) [2] -- the
    largest l with min_len <= l <= min(|A|, |B|) such that the last l bases of A equal the
    first l of B; rows [a, b, strand, l] sorted."""
    rs = reads(text)
    out = []
    for a, ra in enumerate(rs):
        for b, rb in enumerate(rs):
            if a == b:
                continue
            for o, (A, B) in enumerate(((ra, rb), (ra, revcomp(rb)), (revcomp(ra), rb))):
                for l in range(min(len(A), len(B)), min_len - 1, -1):
                    if l > 0 and A[len(A) - l:] == B[:l]:
                        out.append([a, b, o, l])
                        break
    return out
