"""CPU oracle for the suffix-array / LCP / overlap path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline leg
are the only callers.  Nothing in the GPU library imports, links or runs this package, and it
imports nothing from the library.

``saoracle.c`` holds the plain definitions (see its header); ``brute.py`` holds pure-Python
literal definitions for tiny inputs, used to pin the C code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "saoracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile saoracle.c with gcc (-O2, OpenMP) into liboracle.so next to it."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I32 = ctypes.c_int32
        lib.oracle_sa.argtypes = [P, I64, P, ctypes.c_int]
        lib.oracle_sa.restype = ctypes.c_int
        lib.oracle_lcp.argtypes = [P, I64, P, P, ctypes.c_int]
        lib.oracle_lcp.restype = ctypes.c_int
        lib.oracle_overlaps_brute.argtypes = [P, I64, I32, P, I64, ctypes.c_int]
        lib.oracle_overlaps_brute.restype = I64
        lib.oracle_overlaps_indexed.argtypes = [P, I64, I32, P, I64, ctypes.c_int]
        lib.oracle_overlaps_indexed.restype = I64
        lib.oracle_suffix_cmp.argtypes = [P, I64, I64, I64]
        lib.oracle_suffix_cmp.restype = ctypes.c_int
        lib.oracle_lcp_pair.argtypes = [P, I64, I64, I64]
        lib.oracle_lcp_pair.restype = I64
        lib.oracle_num_reads.argtypes = [P, I64]
        lib.oracle_num_reads.restype = I64
        lib.oracle_check_adjacent.argtypes = [P, I64, P, P, P, I64, P, ctypes.c_int]
        lib.oracle_check_adjacent.restype = I64
        lib.oracle_check_range.argtypes = [P, I64, P, P, I64, I64, P, ctypes.c_int]
        lib.oracle_check_range.restype = I64
        lib.oracle_lookup.argtypes = [P, I64, P, P, I64, P, ctypes.c_int]
        lib.oracle_lookup.restype = ctypes.c_int
        _lib = lib
    return _lib


def _threads(nthreads, work=None):
    """Thread count for one call: the caller's, else OMP_NUM_THREADS (else every core), but one
    thread for inputs too small to share (a thread team per tiny call costs more than the work,
    and under several test processes its waiting threads crowd out the others)."""
    if nthreads is None:
        if work is not None and work < (1 << 16):
            return 1
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return max(1, int(nthreads))


def _text(text) -> np.ndarray:
    if isinstance(text, (bytes, bytearray)):
        text = np.frombuffer(bytes(text), dtype=np.uint8)
    t = np.ascontiguousarray(text, dtype=np.uint8)
    if t.size == 0 or t[-1] != ord("$"):
        raise ValueError("text must be non-empty and end with '$'")
    return t


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def suffix_array(text, nthreads=None) -> np.ndarray:
    t = _text(text)
    sa = np.empty(t.size, dtype=np.int32)
    rc = _load().oracle_sa(_ptr(t), t.size, _ptr(sa), _threads(nthreads, t.size))
    if rc != 0:
        raise RuntimeError(f"oracle_sa failed ({rc})")
    return sa


def lcp_array(text, sa, nthreads=None) -> np.ndarray:
    t = _text(text)
    sa = np.ascontiguousarray(sa, dtype=np.int32)
    lcp = np.empty(t.size, dtype=np.int32)
    rc = _load().oracle_lcp(_ptr(t), t.size, _ptr(sa), _ptr(lcp), _threads(nthreads, t.size))
    if rc != 0:
        raise RuntimeError(f"oracle_lcp failed ({rc})")
    return lcp


def _overlaps(fn, text, min_len, nthreads):
    t = _text(text)
    nt = _threads(nthreads, t.size)
    total = fn(_ptr(t), t.size, int(min_len), None, 0, nt)
    if total < 0:
        raise ValueError("bad text or min_len")
    out = np.empty((max(total, 1), 3), dtype=np.int32)
    total2 = fn(_ptr(t), t.size, int(min_len), _ptr(out), total, nt)
    assert total2 == total
    return out[:total]


def overlaps_brute(text, min_len, nthreads=None) -> np.ndarray:
    """All ordered read pairs by the literal definition: (k, 3) int32 rows (a, b, l)."""
    return _overlaps(_load().oracle_overlaps_brute, text, min_len, nthreads)


def overlaps(text, min_len, nthreads=None) -> np.ndarray:
    """Exact seed-and-verify overlaps (same result as overlaps_brute): (k, 3) int32."""
    return _overlaps(_load().oracle_overlaps_indexed, text, min_len, nthreads)


def suffix_cmp(text, p, q) -> int:
    t = _text(text)
    return int(_load().oracle_suffix_cmp(_ptr(t), t.size, int(p), int(q)))


def lcp_pair(text, p, q) -> int:
    t = _text(text)
    return int(_load().oracle_lcp_pair(_ptr(t), t.size, int(p), int(q)))


def num_reads(text) -> int:
    t = _text(text)
    return int(_load().oracle_num_reads(_ptr(t), t.size))


def check_adjacent(text, sa, lcp, idx, nthreads=None):
    """Sampled check at any size: for each i in idx, suffix sa[i-1] < suffix sa[i] and (if lcp
    is given) lcp[i] equals the direct common prefix.  Returns (n_bad, first_bad_index)."""
    t = _text(text)
    sa = np.ascontiguousarray(sa, dtype=np.int32)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    lp = None
    if lcp is not None:
        lcp = np.ascontiguousarray(lcp, dtype=np.int32)
        lp = _ptr(lcp)
    first = ctypes.c_int64(-1)
    bad = _load().oracle_check_adjacent(_ptr(t), t.size, _ptr(sa), lp, _ptr(idx), idx.size,
                                        ctypes.byref(first), _threads(nthreads, idx.size))
    return int(bad), int(first.value)


def check_all(text, sa, lcp, lo=1, hi=None, nthreads=None):
    """Exhaustive check of the adjacent pairs with index in [lo, hi) (default: all of them):
    suffix sa[i-1] < suffix sa[i], and lcp[i] (if lcp is given) equals the direct common prefix.
    With sa a permutation (checked by the caller) this pins sa and lcp element by element.
    Returns (n_bad, first_bad_index)."""
    t = _text(text)
    sa = np.ascontiguousarray(sa, dtype=np.int32)
    if sa.size != t.size:
        raise ValueError("sa and text differ in length")
    lp = None
    if lcp is not None:
        lcp = np.ascontiguousarray(lcp, dtype=np.int32)
        lp = _ptr(lcp)
    hi = t.size if hi is None else int(hi)
    first = ctypes.c_int64(-1)
    bad = _load().oracle_check_range(_ptr(t), t.size, _ptr(sa), lp, int(lo), hi,
                                     ctypes.byref(first), _threads(nthreads, hi - int(lo)))
    return int(bad), int(first.value)


def lookup(text, patterns, nthreads=None) -> np.ndarray:
    """SA interval [lo, hi) of the suffixes that start with each pattern, from the definition
    over text positions (no suffix array): (k, 2) int64.  `patterns` is a list of byte strings
    without separators."""
    t = _text(text)
    pats = [bytes(p) for p in patterns]
    off = np.zeros(len(pats) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(p) for p in pats])
    buf = np.frombuffer(b"".join(pats) + b"\0", dtype=np.uint8).copy()
    out = np.zeros((max(len(pats), 1), 2), dtype=np.int64)
    rc = _load().oracle_lookup(_ptr(t), t.size, _ptr(buf), _ptr(off), len(pats), _ptr(out),
                               _threads(nthreads, t.size * max(len(pats), 1)))
    if rc != 0:
        raise ValueError("pattern holds a separator, or bad text")
    return out[: len(pats)]


_COMP = np.arange(256, dtype=np.uint8)
for _x, _y in ((b"A", b"T"), (b"C", b"G"), (b"G", b"C"), (b"T", b"A")):
    _COMP[_x[0]] = _y[0]


def overlaps_rc(text, min_len, nthreads=None) -> np.ndarray:
    """Overlaps on both strands: (k, 4) int32 rows (a, b, strand, l), a != b, sorted by
    (a, b, strand): strand 0 = a then b, 1 = a then the reverse complement of b, 2 = the reverse
    complement of a then b.  Computed as the forward overlaps of the text followed by every
    read's reverse complement (read m+k is the reverse complement of read m-1-k); a row of two
    reverse complements repeats a strand-0 row and is dropped."""
    t = _text(text)
    m = int((t == ord("$")).sum())
    doubled = np.concatenate([t, _COMP[t[:-1][::-1]], np.array([ord("$")], dtype=np.uint8)])
    rows = overlaps(doubled, min_len, nthreads).astype(np.int64)
    x, y, l = rows[:, 0], rows[:, 1], rows[:, 2]
    xf, yf = x < m, y < m
    a = np.where(xf, x, 2 * m - 1 - x)
    b = np.where(yf, y, 2 * m - 1 - y)
    strand = np.where(xf, np.where(yf, 0, 1), 2)
    keep = (xf | yf) & (a != b)
    out = np.stack([a, b, strand, l], axis=1)[keep]
    order = np.lexsort((out[:, 2], out[:, 1], out[:, 0]))
    return out[order].astype(np.int32)
