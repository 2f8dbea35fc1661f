"""Checks shared by the oracle tests and the GPU parity tests.

Each check states a property the paper's definitions fix (a suffix array is a permutation in
suffix order, an LCP entry is a common-prefix length, an overlap is a string equality that no
longer length satisfies), written independently of both the oracle and the GPU library.
"""
from __future__ import annotations

import numpy as np

SEP = ord("$")


def separators(text: np.ndarray) -> np.ndarray:
    return np.flatnonzero(np.asarray(text) == SEP)


def read_table(text: np.ndarray):
    """(start, length) of each read; read id = order of its separator."""
    ends = separators(text)
    starts = np.concatenate([[0], ends[:-1] + 1]) if ends.size else np.zeros(0, np.int64)
    return starts.astype(np.int64), (ends - starts).astype(np.int64)


def assert_sa_basic(text, sa):
    """SA is a permutation of 0..n-1 and begins with the separators in read order."""
    text = np.asarray(text)
    sa = np.asarray(sa)
    n = text.size
    assert sa.shape == (n,), (sa.shape, n)
    assert sa.min() >= 0 and sa.max() < n
    seen = np.bincount(sa.astype(np.int64), minlength=n)
    assert np.all(seen == 1), "SA is not a permutation"
    seps = separators(text)
    assert np.array_equal(sa[: seps.size], seps), "separators must sort first, in read order"


def isa_of(sa) -> np.ndarray:
    sa = np.asarray(sa, dtype=np.int64)
    isa = np.empty_like(sa)
    isa[sa] = np.arange(sa.size)
    return isa


def assert_kasai_property(text, sa, lcp):
    """Within a read, the LCP of suffix p+1 with its predecessor is at least that of p minus
    one (the permuted-LCP property Kasai's algorithm rests on)."""
    text = np.asarray(text)
    isa = isa_of(sa)
    plcp = np.asarray(lcp, dtype=np.int64)[isa]
    same_read = text[:-1] != SEP
    ok = plcp[1:] >= plcp[:-1] - 1
    assert np.all(ok[same_read]), "PLCP[p+1] >= PLCP[p]-1 violated"


def assert_lcp_bounds(text, sa, lcp):
    """lcp[0] == 0 and lcp[i] <= min(L(sa[i-1]), L(sa[i])) where L is the distance to the
    next separator."""
    text = np.asarray(text)
    n = text.size
    nxt = np.empty(n, dtype=np.int64)
    seps = separators(text)
    idx = np.searchsorted(seps, np.arange(n))
    nxt[:] = seps[idx]
    L = nxt - np.arange(n)
    sa = np.asarray(sa, dtype=np.int64)
    lcp = np.asarray(lcp, dtype=np.int64)
    assert lcp[0] == 0
    assert np.all(lcp[1:] <= np.minimum(L[sa[:-1]], L[sa[1:]]))


def assert_overlaps_valid(text, ovl, min_len):
    """Every triple is a real suffix/prefix equality of length >= min_len, a != b, no longer
    overlap exists (maximality), and rows are sorted by (a, b) without duplicates."""
    text = np.asarray(text)
    starts, lens = read_table(text)
    ovl = np.asarray(ovl).reshape(-1, 3)
    raw = text.tobytes()
    if ovl.shape[0]:
        key = ovl[:, 0].astype(np.int64) * (1 << 32) + ovl[:, 1]
        assert np.all(np.diff(key) > 0), "rows must be strictly sorted by (a, b)"
    for a, b, l in ovl.tolist():
        assert a != b and l >= min_len
        la, lb = int(lens[a]), int(lens[b])
        assert l <= min(la, lb)
        sa_, sb_ = int(starts[a]), int(starts[b])
        ra = raw[sa_:sa_ + la]
        rb = raw[sb_:sb_ + lb]
        assert ra[la - l:] == rb[:l], (a, b, l)
        for l2 in range(l + 1, min(la, lb) + 1):
            assert ra[la - l2:] != rb[:l2], ("not maximal", a, b, l, l2)


def positional_overlaps(starts, read_len, min_len):
    """Ground truth for error-free equal-length reads: b starts d >= 0 bases after a and
    d <= L - min_len gives the overlap L - d (ties d = 0 give both directions)."""
    starts = np.asarray(starts, dtype=np.int64)
    m = starts.size
    out = []
    for a in range(m):
        d = starts - starts[a]
        ok = (d >= 0) & (d <= read_len - min_len)
        ok[a] = False
        for b in np.flatnonzero(ok):
            out.append((a, int(b), int(read_len - d[b])))
    out.sort()
    return np.asarray(out, dtype=np.int32).reshape(-1, 3)


def positional_overlaps_ragged(starts, lengths, min_len):
    """Ground truth for error-free reads of any lengths cut from a random sequence: a read a
    (covering [s_a, e_a)) overlaps b with l = e_a - s_b exactly when s_a <= s_b, e_a <= e_b
    and l >= min_len (a's suffix and b's prefix are then the same stretch of the sequence);
    longer chance matches are ignored, as for positional_overlaps.  Rows sorted by (a, b)."""
    starts = np.asarray(starts, dtype=np.int64)
    ends = starts + np.asarray(lengths, dtype=np.int64)
    order = np.argsort(starts, kind="stable")
    ss = starts[order]
    lo = np.searchsorted(ss, starts, "left")
    hi = np.searchsorted(ss, ends - min_len, "right")
    cnt = np.maximum(hi - lo, 0)
    total = int(cnt.sum())
    a = np.repeat(np.arange(starts.size, dtype=np.int64), cnt)
    first = np.repeat(lo, cnt)
    k = np.arange(total, dtype=np.int64) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    b = order[first + k]
    ell = ends[a] - starts[b]
    keep = (a != b) & (ends[a] <= ends[b]) & (ell >= min_len)
    a, b, ell = a[keep], b[keep], ell[keep]
    o = np.lexsort((b, a))
    return np.stack([a[o], b[o], ell[o]], axis=1).astype(np.int32)


def reversed_reads_text(text) -> np.ndarray:
    """Same reads, each written backwards, separators in place."""
    text = np.asarray(text).copy()
    starts, lens = read_table(text)
    for s, L in zip(starts.tolist(), lens.tolist()):
        text[s:s + L] = text[s:s + L][::-1].copy()
    return text


def swap_pairs(ovl) -> np.ndarray:
    """(a, b, l) -> (b, a, l), re-sorted by the new (a, b)."""
    ovl = np.asarray(ovl).reshape(-1, 3)
    sw = ovl[:, [1, 0, 2]]
    order = np.lexsort((sw[:, 1], sw[:, 0]))
    return sw[order]


def positional_overlaps_rc(starts, strands, read_len, min_len):
    """Ground truth on both strands for error-free equal-length reads: read x covers genome
    [s_x, s_x + L) in orientation d_x (+1 forward, -1 reverse).  For a != b and each way of
    meeting -- (A, B) = (a, b), (a, rc b), (rc a, b) -- A's suffix meets B's prefix when A and
    B run the same way and B starts 0 <= e <= L - min_len bases after A along that direction,
    overlap L - e."""
    starts = np.asarray(starts, dtype=np.int64)
    d = np.where(np.asarray(strands) == 1, -1, 1)
    m = starts.size
    out = []
    for a in range(m):
        for b in range(m):
            if a == b:
                continue
            for o, (da, db) in enumerate(((d[a], d[b]), (d[a], -d[b]), (-d[a], d[b]))):
                if da != db:
                    continue
                e = (starts[b] - starts[a]) * da
                if 0 <= e <= read_len - min_len:
                    out.append((a, b, o, int(read_len - e)))
    out.sort()
    return np.asarray(out, dtype=np.int32).reshape(-1, 4)
