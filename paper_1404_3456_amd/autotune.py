"""Measured choice of radix-sort launch parameters (digit width, tile shape) and, for batched
builds, of set packing, with a JSON cache.

Every candidate runs the real build on the caller's text on the current GPU; the fastest (best
of `reps` timed runs after one warm-up) wins.  All candidates give byte-identical results (the
suffix array is unique), so the choice only affects speed.  The cache key is the device name,
the text length rounded to a power of two and the number of texts rounded likewise.
"""
from __future__ import annotations

import json
import math
import os
import time

from . import _abi

DEFAULT_CACHE = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")),
                             "saasm", "autotune.json")

# (digit_bits, block_threads, items_per_thread)
TILE_CANDIDATES = [(8, 1024, 16), (9, 1024, 16), (8, 512, 16), (9, 512, 16), (8, 256, 16),
                   (8, 512, 8), (11, 512, 16), (4, 1024, 16)]


def _bucket(x: int) -> int:
    return 1 << max(0, int(math.ceil(math.log2(max(1, x)))))


def cache_key(n: int, n_sets: int) -> str:
    import torch
    name = torch.cuda.get_device_properties(torch.cuda.current_device()).name
    return f"{name}|n{_bucket(n)}|sets{_bucket(n_sets)}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(text, set_off=None, candidates=None, seg_packs=(0,), reps=2, cache_path=DEFAULT_CACHE,
             use_cache=True, log=None):
    """Returns (Tuning, report).  `text` is a device uint8 tensor; `set_off` (host int64 offsets)
    selects the batched build.  `seg_packs` lists packing limits to try (batched only)."""
    import torch
    n = int(text.numel())
    n_sets = 1 if set_off is None else len(set_off) - 1
    key = cache_key(n, n_sets)
    cache = _load(cache_path) if (use_cache and cache_path) else {}
    if use_cache and key in cache:
        c = cache[key]
        return _abi.Tuning(*c["tuning"]), {"cached": True, "key": key, **c}
    candidates = candidates or TILE_CANDIDATES
    packs = seg_packs if set_off is not None else (0,)
    results = []
    for d, b, i in candidates:
        for pack in packs:
            tu = _abi.Tuning(d, b, i, int(pack))

            def run():
                if set_off is None:
                    _abi.sa_build(text, isa=True, tuning=tu)
                else:
                    _abi.sa_build_batched(text, set_off, isa=True, tuning=tu, use_graph=False)

            run()
            torch.cuda.synchronize()
            best = math.inf
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                run()
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            results.append({"tuning": [d, b, i, int(pack)], "ms": round(best * 1e3, 3)})
            if log:
                log(f"autotune {key}: {results[-1]}")
    best = min(results, key=lambda r: r["ms"])
    entry = {"tuning": best["tuning"], "ms": best["ms"], "tried": results}
    if cache_path:
        cache = _load(cache_path)
        cache[key] = entry
        _save(cache_path, cache)
    return _abi.Tuning(*best["tuning"]), {"cached": False, "key": key, **entry}
