"""ctypes marshalling for libsaasm.so (see include/saasm.h for every argument's meaning)."""
from __future__ import annotations

import ctypes
import dataclasses
import os

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(HERE, "libsaasm.so")

SA_OK = 0
SA_PENDING = 1
SA_ERR_INVALID = -1
SA_ERR_ALPHABET = -2
SA_ERR_TOO_LARGE = -3
SA_ERR_NOMEM = -4
SA_ERR_CAPACITY = -5
SA_ERR_HIP = -6
SA_ERR_NOTFOUND = -7
ASM_BORROW = 1

_lib = None


class SaasmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"saasm error {code}: {msg}")
        self.code = code


class _AsmResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("n_overlaps", ctypes.c_int64), ("sa", ctypes.c_void_p), ("isa", ctypes.c_void_p),
                ("lcp", ctypes.c_void_p), ("ovl", ctypes.c_void_p), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class _Tuning(ctypes.Structure):
    _fields_ = [("digit_bits", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("items_per_thread", ctypes.c_int32), ("seg_pack", ctypes.c_int32)]


@dataclasses.dataclass
class Tuning:
    digit_bits: int = 0
    block_threads: int = 0
    items_per_thread: int = 0
    seg_pack: int = 0

    def c(self):
        return _Tuning(self.digit_bits, self.block_threads, self.items_per_thread, self.seg_pack)


def lib_path() -> str:
    return _LIB


def load():
    """Load libsaasm.so (built in-tree by paper_1404_3456_amd.build); raises when missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        raise ImportError(f"{_LIB} is missing: build it with `python -m paper_1404_3456_amd.build`")
    # torch first: its bundled HIP runtime carries the soname the library links against, so the
    # library binds to that one copy.  Opened before torch, the library would pull the system
    # runtime in beside torch's, and tensors, streams and the server's threads would then be
    # split over two HIP (and two HSA) runtimes in one process.
    _torch()
    lib = ctypes.CDLL(_LIB)
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    TP = ctypes.POINTER(_Tuning)
    sig = {
        "sa_version": ([], ctypes.c_char_p),
        "sa_last_error": ([], ctypes.c_char_p),
        "sa_packed_words": ([I64], I64),
        "sa_sepmask_words": ([I64], I64),
        "sa_pack_ws_bytes": ([I64], I64),
        "sa_pack": ([P, I64, P, P, P, I64, P, P, I64, P], ctypes.c_int),
        "sa_sort_ws_bytes": ([I64, TP], I64),
        "sa_sort_pairs": ([P, P, I64, I32, I32, P, I64, TP, P], ctypes.c_int),
        "sa_build_ws_bytes": ([I64, TP], I64),
        "sa_build": ([P, I64, P, P, P, I64, TP, P, P], ctypes.c_int),
        "sa_build_dc3_ws_bytes": ([I64, TP], I64),
        "sa_build_dc3": ([P, I64, P, P, P, I64, TP, P, P], ctypes.c_int),
        "sa_build_batched_ws_bytes": ([I64, I32, P, TP], I64),
        "sa_build_batched": ([P, I64, P, I32, P, P, P, P, I64, TP, I32, P, P], ctypes.c_int),
        "sa_workspace_bytes": ([I64, I64], I64),
        "sa_lcp_status": ([P, P], ctypes.c_int),
        "sa_lcp_ws_bytes": ([I64], I64),
        "sa_lookup_ws_bytes": ([I64, I64], I64),
        "sa_reconstruct": ([P, I64, P, P, P, P, P, I64, P, I64], ctypes.c_int),
        "sa_overlap_path": ([P, I64, P, I64, I32, P, P, P, I64, P], ctypes.c_int),
        "sa_revcomp_text": ([P, I64, P, P, P, I64, P], ctypes.c_int),
        "sa_strand_rows_ws_bytes": ([I64, I64], I64),
        "sa_strand_rows": ([P, I64, I64, P, I64, P, P, I64, P], ctypes.c_int),
        "sa_lookup": ([P, I64, P, P, P, I64, ctypes.c_int32, P, P, I64, P], ctypes.c_int),
        "sa_lcp": ([P, I64, P, P, P, P, I64, P], ctypes.c_int),
        "sa_lcp_noalloc": ([P, I64, P, P, P, P], ctypes.c_int),
        "sa_lcp_noalloc_max_n": ([], I64),
        "sa_lcp_set_chunk": ([I32], ctypes.c_int),
        "sa_lcp_plcp_min": ([I64], I64),
        "sa_overlaps_ws_bytes": ([I64, I64, I64], I64),
        "sa_overlaps": ([P, I64, P, P, P, I32, P, I64, P, P, I64, P, P], ctypes.c_int),
        "sa_timing_enable": ([I32], ctypes.c_int),
        "sa_timing_reset": ([], ctypes.c_int),
        "sa_timing_get": ([ctypes.c_char_p, P, P, P], ctypes.c_int),
        "sa_timing_items": ([ctypes.c_char_p, P], ctypes.c_int),
        "sa_copy_u32": ([P, P, I64, P], ctypes.c_int),
        "asm_server_create": ([P, I64, I32, I32, I32, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
        "asm_submit": ([P, P, I64, I32, I32, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "asm_poll": ([P, ctypes.c_uint64, ctypes.POINTER(_AsmResult)], ctypes.c_int),
        "asm_release": ([P, ctypes.c_uint64], ctypes.c_int),
        "asm_server_stats": ([P, P], ctypes.c_int),
        "asm_server_fail_alloc_after": ([P, I32], ctypes.c_int),
        "asm_server_destroy": ([P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def sa_version() -> str:
    return load().sa_version().decode()


def sa_last_error() -> str:
    return load().sa_last_error().decode()


def _check(rc: int):
    if rc != SA_OK:
        raise SaasmError(rc, sa_last_error())


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _tune(tuning):
    if tuning is None:
        return None
    if isinstance(tuning, dict):
        tuning = Tuning(**tuning)
    return ctypes.byref(tuning.c())


def _dev_text(text):
    torch = _torch()
    if not isinstance(text, torch.Tensor):
        import numpy as np
        text = torch.from_numpy(np.ascontiguousarray(text, dtype=np.uint8))
    if text.dtype != torch.uint8:
        raise TypeError("text must be uint8")
    if not text.is_cuda:
        text = text.cuda()
    return text.contiguous()


def _ws(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# ---- entry points --------------------------------------------------------------------------

def sa_build_ws_bytes(n: int, tuning=None) -> int:
    return int(load().sa_build_ws_bytes(n, _tune(tuning)))


def sa_build_dc3_ws_bytes(n: int, tuning=None) -> int:
    return int(load().sa_build_dc3_ws_bytes(n, _tune(tuning)))


def sa_lcp_ws_bytes(n: int) -> int:
    return int(load().sa_lcp_ws_bytes(n))


def sa_overlaps_ws_bytes(n: int, m: int = 0, candidates: int = 0) -> int:
    return int(load().sa_overlaps_ws_bytes(n, m, candidates))


def sa_sort_ws_bytes(n: int, tuning=None) -> int:
    return int(load().sa_sort_ws_bytes(n, _tune(tuning)))


def sa_pack(text, with_read_ends: bool = True, stream=None):
    """Returns (packed uint32, sepmask uint32, read_end int32 or None)."""
    torch = _torch()
    lib = load()
    t = _dev_text(text)
    n = t.numel()
    packed = torch.empty(int(lib.sa_packed_words(n)), dtype=torch.int32, device=t.device)
    sepmask = torch.empty(int(lib.sa_sepmask_words(n)), dtype=torch.int32, device=t.device)
    m = ctypes.c_int64(0)
    read_end = torch.empty(max(n, 1), dtype=torch.int32, device=t.device) if with_read_ends else None
    cap = n if with_read_ends else 0
    ws = _ws(int(lib.sa_pack_ws_bytes(n)), t.device)
    _check(lib.sa_pack(_ptr(t), n, _ptr(packed), _ptr(sepmask), _ptr(read_end), cap,
                       ctypes.byref(m), _ptr(ws), ws.numel(), _stream(stream)))
    if read_end is not None:
        read_end = read_end[: m.value]
    return packed, sepmask, read_end


def sa_sort_pairs(keys, vals, bit_lo: int = 0, bit_hi: int = 64, tuning=None, stream=None):
    """Stable in-place sort of (keys int64/uint64, vals int32/uint32) by key bits [lo, hi)."""
    lib = load()
    n = keys.numel()
    if vals.numel() != n:
        raise ValueError("keys and vals differ in length")
    if not (keys.is_contiguous() and vals.is_contiguous()):
        raise ValueError("keys and vals must be contiguous")
    if keys.element_size() != 8 or vals.element_size() != 4:
        raise TypeError("keys must be 64-bit and vals 32-bit")
    wsb = sa_sort_ws_bytes(n, tuning)
    ws = _ws(wsb, keys.device)
    _check(lib.sa_sort_pairs(_ptr(keys), _ptr(vals), n, bit_lo, bit_hi, _ptr(ws), ws.numel(),
                             _tune(tuning), _stream(stream)))
    return keys, vals


def sa_build(text, isa: bool = True, tuning=None, stream=None, return_rounds: bool = False):
    """Suffix array (and inverse) of a '$'-separated text on the GPU."""
    torch = _torch()
    lib = load()
    t = _dev_text(text)
    n = t.numel()
    sa = torch.empty(n, dtype=torch.int32, device=t.device)
    isa_t = torch.empty(n, dtype=torch.int32, device=t.device) if isa else None
    wsb = sa_build_ws_bytes(n, tuning)
    if wsb < 0:
        raise SaasmError(SA_ERR_INVALID, "bad size or tuning")
    ws = _ws(wsb, t.device)
    rounds = ctypes.c_int32(0)
    _check(lib.sa_build(_ptr(t), n, _ptr(sa), _ptr(isa_t), _ptr(ws), ws.numel(), _tune(tuning),
                        ctypes.byref(rounds), _stream(stream)))
    if return_rounds:
        return sa, isa_t, int(rounds.value)
    return sa, isa_t


def sa_build_dc3(text, isa: bool = True, tuning=None, stream=None, return_levels: bool = False):
    """The same suffix array (and inverse) by the skew recursion (sa_build_dc3)."""
    torch = _torch()
    lib = load()
    t = _dev_text(text)
    n = t.numel()
    sa = torch.empty(n, dtype=torch.int32, device=t.device)
    isa_t = torch.empty(n, dtype=torch.int32, device=t.device) if isa else None
    wsb = sa_build_dc3_ws_bytes(n, tuning)
    if wsb < 0:
        raise SaasmError(SA_ERR_INVALID, "bad size or tuning")
    ws = _ws(wsb, t.device)
    levels = ctypes.c_int32(0)
    _check(lib.sa_build_dc3(_ptr(t), n, _ptr(sa), _ptr(isa_t), _ptr(ws), ws.numel(),
                            _tune(tuning), ctypes.byref(levels), _stream(stream)))
    if return_levels:
        return sa, isa_t, int(levels.value)
    return sa, isa_t


def sa_build_batched_ws_bytes(n: int, n_sets: int, tuning=None, set_off=None) -> int:
    import numpy as np
    off = None if set_off is None else np.ascontiguousarray(set_off, dtype=np.int64)
    ptr = None if off is None else off.ctypes.data_as(ctypes.c_void_p)
    return int(load().sa_build_batched_ws_bytes(n, n_sets, ptr, _tune(tuning)))


def sa_build_batched(text, set_off, isa: bool = True, tuning=None, use_graph: bool = False,
                     stream=None, return_rounds: bool = False, lcp: bool = False):
    """Suffix arrays of many texts laid end to end.  `set_off` (host, int64, n_sets+1) bounds
    text s as text[set_off[s]:set_off[s+1]].  Returns (sa, isa) in concatenated coordinates:
    sa[set_off[s]:set_off[s+1]] is the suffix array of text s; with lcp=True, (sa, isa, lcp)
    where lcp is computed inside the same call (its status is checked).  use_graph replays the
    doubling rounds from a captured hipGraph instead of the host-driven loop (same result)."""
    import numpy as np
    torch = _torch()
    lib = load()
    t = _dev_text(text)
    n = t.numel()
    off = np.ascontiguousarray(set_off, dtype=np.int64)
    n_sets = off.size - 1
    sa = torch.empty(n, dtype=torch.int32, device=t.device)
    isa_t = torch.empty(n, dtype=torch.int32, device=t.device) if isa else None
    wsb = sa_build_batched_ws_bytes(n, n_sets, tuning, off)
    if wsb < 0:
        raise SaasmError(SA_ERR_INVALID, "bad size, set count or tuning")
    ws = _ws(wsb, t.device)
    rounds = ctypes.c_int32(0)
    lcp_t = torch.empty(n, dtype=torch.int32, device=t.device) if lcp else None
    _check(lib.sa_build_batched(_ptr(t), n, off.ctypes.data_as(ctypes.c_void_p), n_sets, _ptr(sa),
                                _ptr(isa_t), _ptr(lcp_t), _ptr(ws), ws.numel(), _tune(tuning),
                                1 if use_graph else 0, ctypes.byref(rounds), _stream(stream)))
    if lcp:
        _check(lib.sa_lcp_status(_ptr(lcp_t), _stream(stream)))
    res = (sa, isa_t, lcp_t) if lcp else (sa, isa_t)
    if return_rounds:
        return (*res, int(rounds.value))
    return res


def sa_lcp(text, sa, isa, stream=None, check: bool = False):
    """LCP array (asynchronous).  A failure only the device sees is left in lcp[0] as a
    negative status; check=True waits for it (sa_lcp_status) and raises."""
    torch = _torch()
    lib = load()
    t = _dev_text(text)
    n = t.numel()
    lcp = torch.empty(n, dtype=torch.int32, device=t.device)
    ws = _ws(sa_lcp_ws_bytes(n), t.device)
    _check(lib.sa_lcp(_ptr(t), n, _ptr(sa), _ptr(isa), _ptr(lcp), _ptr(ws), ws.numel(),
                      _stream(stream)))
    if check:
        sa_lcp_status(lcp, stream)
    return lcp


def sa_lcp_noalloc(text, sa, isa, lcp, stream=None, check: bool = False):
    """sa_lcp into the caller's `lcp` tensor with the library's own device scratch (no
    allocation; n <= sa_lcp_noalloc_max_n())."""
    lib = load()
    t = _dev_text(text)
    _check(lib.sa_lcp_noalloc(_ptr(t), t.numel(), _ptr(sa), _ptr(isa), _ptr(lcp), _stream(stream)))
    if check:
        sa_lcp_status(lcp, stream)
    return lcp


def sa_lcp_noalloc_max_n() -> int:
    return int(load().sa_lcp_noalloc_max_n())


def sa_lcp_status(lcp, stream=None):
    """Waits for the stream and raises SaasmError when sa_lcp left a failure in lcp[0]."""
    _check(load().sa_lcp_status(_ptr(lcp), _stream(stream)))


def sa_workspace_bytes(n: int, n_reads_upper: int = 0) -> int:
    return int(load().sa_workspace_bytes(int(n), int(n_reads_upper)))


def sa_path(text, min_len: int, stream=None, ws=None):
    """The whole path -- sa_build, sa_lcp, sa_overlaps -- through one workspace of
    sa_workspace_bytes(n, reads) bytes (allocated here unless `ws` is given): (sa, isa, lcp,
    overlap rows)."""
    torch = _torch()
    lib = load()
    t = _dev_text(text)
    n = t.numel()
    if ws is None:
        ws = _ws(sa_workspace_bytes(n, 0), t.device)
    sa = torch.empty(n, dtype=torch.int32, device=t.device)
    isa_t = torch.empty(n, dtype=torch.int32, device=t.device)
    lcp = torch.empty(n, dtype=torch.int32, device=t.device)
    st = _stream(stream)
    _check(lib.sa_build(_ptr(t), n, _ptr(sa), _ptr(isa_t), _ptr(ws), ws.numel(), None, None, st))
    _check(lib.sa_lcp(_ptr(t), n, _ptr(sa), _ptr(isa_t), _ptr(lcp), _ptr(ws), ws.numel(), st))
    cap = max(n // 64, 1024)
    for _ in range(4):
        out = torch.empty((cap, 3), dtype=torch.int32, device=t.device)
        n_out = ctypes.c_int64(0)
        needed = ctypes.c_int64(0)
        rc = lib.sa_overlaps(_ptr(t), n, _ptr(sa), _ptr(isa_t), _ptr(lcp), int(min_len), _ptr(out),
                             cap, ctypes.byref(n_out), _ptr(ws), ws.numel(), ctypes.byref(needed), st)
        if rc == SA_ERR_CAPACITY and n_out.value > cap:
            cap = int(n_out.value)
            continue
        _check(rc)
        return sa, isa_t, lcp, out[: n_out.value]
    raise SaasmError(SA_ERR_HIP, "sa_path: sizes did not settle")


def sa_lookup_ws_bytes(n: int, pat_total: int) -> int:
    return int(load().sa_lookup_ws_bytes(n, pat_total))


def sa_lookup(text, sa, patterns, stream=None):
    """SA interval [lo, hi) of the suffixes that start with each pattern: (k, 2) int32 device
    tensor.  `patterns` is a list of byte strings, or a pair (device uint8 tensor of the
    concatenated patterns, device int64 tensor of k+1 offsets)."""
    torch = _torch()
    lib = load()
    t = _dev_text(text)
    n = t.numel()
    if isinstance(patterns, tuple):
        buf, off = patterns
    else:
        import numpy as np
        pats = [bytes(p) for p in patterns]
        off_h = np.zeros(len(pats) + 1, dtype=np.int64)
        off_h[1:] = np.cumsum([len(p) for p in pats])
        raw = np.frombuffer(b"".join(pats) or b"\0", dtype=np.uint8).copy()
        buf = torch.from_numpy(raw).to(t.device)
        off = torch.from_numpy(off_h).to(t.device)
    k = off.numel() - 1
    total = int(buf.numel())
    out = torch.empty((max(k, 0), 2), dtype=torch.int32, device=t.device)
    ws = _ws(sa_lookup_ws_bytes(n, total), t.device)
    _check(lib.sa_lookup(_ptr(t), n, _ptr(sa), _ptr(buf), _ptr(off), total, k, _ptr(out),
                         _ptr(ws), ws.numel(), _stream(stream)))
    return out


def sa_reconstruct_host(text, sa, isa, lcp, max_steps: int = 10 ** 7):
    """Cut-and-continue reconstruction (host search) over host numpy arrays: returns
    (sequence bytes, placement order) or None when no reconstruction exists."""
    import numpy as np
    t = np.ascontiguousarray(text, dtype=np.uint8)
    sa = np.ascontiguousarray(sa, dtype=np.int32)
    isa = np.ascontiguousarray(isa, dtype=np.int32)
    lcp = np.ascontiguousarray(lcp, dtype=np.int32)
    m = int((t == ord("$")).sum())
    order = np.empty(max(m, 1), dtype=np.int32)
    rs = np.empty(t.size, dtype=np.uint8)
    rs_len = ctypes.c_int64(0)
    P = ctypes.c_void_p
    rc = load().sa_reconstruct(t.ctypes.data_as(P), t.size, sa.ctypes.data_as(P),
                               isa.ctypes.data_as(P), lcp.ctypes.data_as(P),
                               order.ctypes.data_as(P), rs.ctypes.data_as(P), rs.size,
                               ctypes.byref(rs_len), int(max_steps))
    if rc == SA_ERR_NOTFOUND:
        return None
    _check(rc)
    return bytes(rs[: rs_len.value]), order[:m].tolist()


def sa_overlap_path(text, rows, exact_max_m: int = 16):
    """Maximal-weight Hamiltonian path through the weighted overlap graph (host search over
    host arrays): (order list, total weight, superstring bytes).  `text` holds the fragments
    ('$'-closed), `rows` the (r, 3) overlap rows (numpy, or a tensor copied to the host)."""
    import numpy as np
    t = np.ascontiguousarray(text, dtype=np.uint8)
    if hasattr(rows, "cpu"):
        rows = rows.cpu().numpy()
    rw = np.ascontiguousarray(np.asarray(rows, dtype=np.int32).reshape(-1, 3))
    m = int((t == ord("$")).sum())
    order = np.zeros(max(m, 1), dtype=np.int32)
    weight = ctypes.c_int64(0)
    rs = np.zeros(max(t.size, 1), dtype=np.uint8)
    rs_len = ctypes.c_int64(0)
    P = ctypes.c_void_p
    _check(load().sa_overlap_path(t.ctypes.data_as(P), t.size, rw.ctypes.data_as(P), rw.shape[0],
                                  int(exact_max_m), order.ctypes.data_as(P), ctypes.byref(weight),
                                  rs.ctypes.data_as(P), rs.size, ctypes.byref(rs_len)))
    return order[:m].tolist(), int(weight.value), bytes(rs[: rs_len.value])


def to_host(*tensors):
    """Device tensors to numpy arrays through pinned host buffers (one synchronisation)."""
    torch = _torch()
    outs = []
    for x in tensors:
        h = torch.empty(x.shape, dtype=x.dtype, pin_memory=True)
        h.copy_(x, non_blocking=True)
        outs.append(h)
    torch.cuda.synchronize()
    return [h.numpy() for h in outs]


def sa_reconstruct(text, max_steps: int = 10 ** 7, stream=None):
    """Builds SA, ISA and LCP of the fragment text on the GPU, then runs the host search."""
    t = _dev_text(text)
    sa, isa = sa_build(t, stream=stream)
    lcp = sa_lcp(t, sa, isa, stream=stream)
    t_h, sa_h, isa_h, lcp_h = to_host(t, sa, isa, lcp)
    return sa_reconstruct_host(t_h, sa_h, isa_h, lcp_h, max_steps)


def sa_revcomp_text(text, stream=None):
    """(doubled device text: reads then their reverse complements, number of reads m)."""
    torch = _torch()
    t = _dev_text(text)
    n = t.numel()
    out = torch.empty(2 * n, dtype=torch.uint8, device=t.device)
    ws = _ws(256, t.device)
    m = ctypes.c_int64(0)
    _check(load().sa_revcomp_text(_ptr(t), n, _ptr(out), ctypes.byref(m), _ptr(ws), ws.numel(),
                                  _stream(stream)))
    return out, int(m.value)


def sa_strand_rows(rows, m: int, stream=None):
    """(k, 4) int32 rows (a, b, strand, l) from the (r, 3) overlaps of a doubled text."""
    torch = _torch()
    rows = rows.contiguous()
    r = rows.shape[0]
    ws = _ws(int(load().sa_strand_rows_ws_bytes(r, m)), rows.device)
    cap = max(r, 1)
    out = torch.empty((cap, 4), dtype=torch.int32, device=rows.device)
    n_out = ctypes.c_int64(0)
    _check(load().sa_strand_rows(_ptr(rows), r, m, _ptr(out), cap, ctypes.byref(n_out), _ptr(ws),
                                 ws.numel(), _stream(stream)))
    return out[: n_out.value]


def sa_overlaps_rc(text, min_len: int, stream=None):
    """Overlaps on both strands: (k, 4) int32 device rows (a, b, strand, l), sorted."""
    t2, m = sa_revcomp_text(text, stream=stream)
    sa, isa = sa_build(t2, stream=stream)
    lcp = sa_lcp(t2, sa, isa, stream=stream)
    rows = sa_overlaps(t2, sa, isa, lcp, min_len, stream=stream)
    return sa_strand_rows(rows, m, stream=stream)


def sa_lcp_set_chunk(chunk: int):
    _check(load().sa_lcp_set_chunk(int(chunk)))


def sa_lcp_plcp_min(min_n: int = -1) -> int:
    """Size from which sa_lcp gathers from a position-ordered LCP; min_n >= 0 sets it and
    returns the previous value, min_n < 0 only reads it."""
    return int(load().sa_lcp_plcp_min(int(min_n)))


_ovl_ws_hint = {}


def sa_overlaps(text, sa, isa, lcp, min_len: int, stream=None):
    """(k, 3) int32 device tensor of rows (a, b, l), sorted by (a, b)."""
    torch = _torch()
    lib = load()
    t = _dev_text(text)
    n = t.numel()
    need = max(_ovl_ws_hint.get(n, 0), sa_overlaps_ws_bytes(n, 1, 0))
    cap = max(n // 64, 1024)
    for _ in range(6):
        ws = _ws(need, t.device)
        out = torch.empty((cap, 3), dtype=torch.int32, device=t.device)
        n_out = ctypes.c_int64(0)
        needed = ctypes.c_int64(0)
        rc = lib.sa_overlaps(_ptr(t), n, _ptr(sa), _ptr(isa), _ptr(lcp), int(min_len), _ptr(out),
                             cap, ctypes.byref(n_out), _ptr(ws), ws.numel(), ctypes.byref(needed),
                             _stream(stream))
        if rc == SA_ERR_NOMEM and needed.value > need:
            need = int(needed.value)
            _ovl_ws_hint[n] = need
            continue
        if rc == SA_ERR_CAPACITY and n_out.value > cap:
            cap = int(n_out.value)
            continue
        _check(rc)
        return out[: n_out.value]
    raise SaasmError(SA_ERR_HIP, "sa_overlaps: sizes did not settle")


def sa_timing_enable(on: bool = True):
    _check(load().sa_timing_enable(1 if on else 0))


def sa_timing_reset():
    _check(load().sa_timing_reset())


def sa_timing_get(key: str):
    """(launches, total_ms, total_algorithmic_bytes) for an instrumented kernel key."""
    lib = load()
    L = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    by = ctypes.c_double(0.0)
    rc = lib.sa_timing_get(key.encode(), ctypes.byref(L), ctypes.byref(ms), ctypes.byref(by))
    if rc not in (SA_OK, SA_ERR_NOTFOUND):
        _check(rc)
    return int(L.value), float(ms.value), float(by.value)


def sa_timing_items(key: str) -> float:
    """Summed units of work (suffixes, items, reads) of the timed launches under `key`."""
    v = ctypes.c_double(0.0)
    rc = load().sa_timing_items(key.encode(), ctypes.byref(v))
    if rc not in (SA_OK, SA_ERR_NOTFOUND):
        _check(rc)
    return float(v.value)


def sa_copy_u32(dst, src, stream=None):
    n = src.numel()
    _check(load().sa_copy_u32(_ptr(dst), _ptr(src), n, _stream(stream)))


# ---- assembly-job server ---------------------------------------------------------------------

class AsmServer:
    """Continuous-batching job server over an HBM arena (see asm_server_create in saasm.h).
    Methods mirror the C ABI: asm_submit, asm_poll, asm_release, asm_server_stats."""

    def __init__(self, arena_bytes: int, max_jobs_per_batch: int = 64, workers: int = 2,
                 mode: int = 0, device=None):
        torch = _torch()
        lib = load()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8,
                                 device=device if device is not None else "cuda")
        torch.cuda.synchronize()
        h = ctypes.c_void_p(0)
        _check(lib.asm_server_create(_ptr(self.arena), self.arena.numel(), int(max_jobs_per_batch),
                                     int(workers), int(mode), ctypes.byref(h)))
        self._h = h
        self._lib = lib
        self._borrowed = {}

    def asm_submit(self, text, min_len: int, borrow: bool = False) -> int:
        """Queue a job.  With borrow=True the server reads `text` in place (no copy); the
        binding keeps a reference to it until the job is released."""
        import numpy as np
        t = np.ascontiguousarray(text, dtype=np.uint8)
        jid = ctypes.c_uint64(0)
        _check(self._lib.asm_submit(self._h, t.ctypes.data_as(ctypes.c_void_p), t.size,
                                    int(min_len), ASM_BORROW if borrow else 0, ctypes.byref(jid)))
        if borrow:
            self._borrowed[int(jid.value)] = t
        return int(jid.value)

    def asm_poll(self, job_id: int):
        """None while pending, else a dict with status, times and (on success) device tensors
        that view the server's arena (valid until asm_release)."""
        r = _AsmResult()
        rc = self._lib.asm_poll(self._h, ctypes.c_uint64(job_id), ctypes.byref(r))
        if rc == SA_PENDING:
            return None
        _check(rc)
        out = {"status": r.status, "n": r.n, "m": r.m, "n_overlaps": r.n_overlaps,
               "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done}
        if r.status == SA_OK:
            base = self.arena.data_ptr()

            def view(ptr, count):
                off = ptr - base
                return self.arena[off: off + 4 * count].view(_torch().int32)

            out["sa"] = view(r.sa, r.n)
            out["isa"] = view(r.isa, r.n)
            out["lcp"] = view(r.lcp, r.n)
            out["ovl"] = view(r.ovl, 3 * r.n_overlaps).view(-1, 3) if r.n_overlaps else \
                _torch().zeros((0, 3), dtype=_torch().int32, device=self.arena.device)
        return out

    def asm_release(self, job_id: int):
        _check(self._lib.asm_release(self._h, ctypes.c_uint64(job_id)))
        self._borrowed.pop(int(job_id), None)

    def asm_server_stats(self):
        import numpy as np
        a = np.zeros(6, dtype=np.int64)
        _check(self._lib.asm_server_stats(self._h, a.ctypes.data_as(ctypes.c_void_p)))
        keys = ["batches", "jobs_done", "max_concurrent_batches", "arena_used", "arena_bytes", "queued"]
        return dict(zip(keys, a.tolist()))

    def fail_alloc_after(self, k: int):
        _check(self._lib.asm_server_fail_alloc_after(self._h, int(k)))

    def close(self):
        if self._h:
            _check(self._lib.asm_server_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
