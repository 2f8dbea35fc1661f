"""The C-ABI library loads and exports every symbol include/*.h declares; host-side argument
checks run without a GPU (no compute call is made here)."""
import ctypes

import numpy as np
import glob
import os
import re

import pytest

from paper_1404_3456_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b((?:sa|asm)_\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ["sa_build", "sa_lcp", "sa_overlaps", "sa_pack", "sa_sort_pairs",
                     "sa_last_error", "sa_version", "sa_build_ws_bytes"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_python_binding_names_match_abi():
    import paper_1404_3456_amd as pkg
    for n in ["sa_build", "sa_lcp", "sa_overlaps", "sa_pack", "sa_sort_pairs"]:
        assert callable(getattr(pkg, n))


def test_version_and_workspace_sizes():
    assert "gfx950" in _abi.sa_version()
    assert _abi.sa_build_ws_bytes(1) > 0
    small = _abi.sa_build_ws_bytes(80_400)
    big = _abi.sa_build_ws_bytes(50_100_000)
    assert big > small > 0
    # about 45 bytes per suffix for the default tuning: keys x2, values x2, slots x2, ranks
    assert 30 * 50_100_000 < big < 60 * 50_100_000
    assert _abi.sa_build_ws_bytes(0) == -1
    assert _abi.sa_build_ws_bytes(10, {"digit_bits": 5}) == -1
    assert _abi.sa_lcp_ws_bytes(100) > 0
    assert _abi.sa_overlaps_ws_bytes(100, 1, 0) < _abi.sa_overlaps_ws_bytes(100, 10, 1000)


def test_host_argument_checks_without_gpu():
    lib = _abi.load()
    P = ctypes.c_void_p
    assert lib.sa_build(None, 10, None, None, None, 0, None, None, None) == _abi.SA_ERR_INVALID
    assert "NULL" in _abi.sa_last_error()
    dummy = P(16)
    assert lib.sa_build(dummy, 0, dummy, None, dummy, 1 << 20, None, None, None) == _abi.SA_ERR_INVALID
    assert lib.sa_build(dummy, (1 << 31) - 2, dummy, None, dummy, 1 << 20, None, None, None) == _abi.SA_ERR_TOO_LARGE
    assert lib.sa_build(dummy, 100, dummy, None, dummy, 16, None, None, None) == _abi.SA_ERR_NOMEM
    bad = _abi.Tuning(digit_bits=7).c()
    assert lib.sa_build(dummy, 100, dummy, None, dummy, 1 << 30, ctypes.byref(bad), None, None) == _abi.SA_ERR_INVALID
    assert lib.sa_sort_pairs(dummy, dummy, 10, 5, 5, dummy, 1 << 20, None, None) == _abi.SA_ERR_INVALID
    assert lib.sa_sort_pairs(dummy, dummy, 10, 0, 65, dummy, 1 << 20, None, None) == _abi.SA_ERR_INVALID
    n_out = ctypes.c_int64(0)
    assert lib.sa_overlaps(dummy, 100, dummy, dummy, dummy, 0, dummy, 10, ctypes.byref(n_out),
                           dummy, 1 << 20, None, None) == _abi.SA_ERR_INVALID
    assert lib.sa_lcp(dummy, 100, dummy, None, dummy, dummy, 1 << 20, None) == _abi.SA_ERR_INVALID
    assert lib.sa_lcp_set_chunk(0) == _abi.SA_ERR_INVALID
    assert lib.sa_lcp_set_chunk(3) == _abi.SA_ERR_INVALID
    # the 1024-thread tile needs 16 items and at most 9-bit digits
    for tu in (_abi.Tuning(8, 1024, 8), _abi.Tuning(11, 1024, 16), _abi.Tuning(8, 768, 16)):
        c = tu.c()
        assert lib.sa_build(dummy, 100, dummy, None, dummy, 1 << 30, ctypes.byref(c), None,
                            None) == _abi.SA_ERR_INVALID, tu
    lk = np.zeros(2, dtype=np.int32)
    assert lib.sa_lookup(None, 100, dummy, dummy, dummy, 4, 1, lk.ctypes.data_as(P), dummy,
                         1 << 20, None) == _abi.SA_ERR_INVALID
    assert lib.sa_lookup(dummy, 100, dummy, dummy, dummy, 4, -1, lk.ctypes.data_as(P), dummy,
                         1 << 20, None) == _abi.SA_ERR_INVALID
    assert lib.sa_lookup(dummy, 100, dummy, dummy, dummy, 4, 1, lk.ctypes.data_as(P), dummy,
                         16, None) == _abi.SA_ERR_NOMEM


def test_dc3_host_checks_and_workspace():
    lib = _abi.load()
    dummy = ctypes.c_void_p(16)
    assert lib.sa_build_dc3(None, 10, None, None, None, 0, None, None, None) == _abi.SA_ERR_INVALID
    assert lib.sa_build_dc3(dummy, 0, dummy, None, dummy, 1 << 20, None, None, None) == _abi.SA_ERR_INVALID
    assert lib.sa_build_dc3(dummy, (1 << 31) - 2, dummy, None, dummy, 1 << 20, None, None,
                            None) == _abi.SA_ERR_TOO_LARGE
    assert lib.sa_build_dc3(dummy, 100, dummy, None, dummy, 16, None, None, None) == _abi.SA_ERR_NOMEM
    assert "workspace" in _abi.sa_last_error()
    bad = _abi.Tuning(digit_bits=7).c()
    assert lib.sa_build_dc3(dummy, 100, dummy, None, dummy, 1 << 30, ctypes.byref(bad), None,
                            None) == _abi.SA_ERR_INVALID
    assert _abi.sa_build_dc3_ws_bytes(0) == -1
    assert _abi.sa_build_dc3_ws_bytes(1) > 0
    big = _abi.sa_build_dc3_ws_bytes(50_100_000)
    # per suffix: ranks, samples and name strings over the shrinking levels, the sort buffers
    # for two thirds of the suffixes and a 16-byte comparison record
    assert 40 * 50_100_000 < big < 80 * 50_100_000


def test_lcp_plcp_setting_and_workspace():
    default = _abi.sa_lcp_plcp_min(-1)
    assert default == 1 << 26
    small = _abi.sa_lcp_ws_bytes(1000)
    assert _abi.sa_lcp_plcp_min(0) == default
    try:
        assert _abi.sa_lcp_ws_bytes(1000) >= small + 4000  # room for the position-ordered LCP
    finally:
        assert _abi.sa_lcp_plcp_min(default) == 0
    assert _abi.sa_lcp_ws_bytes(1000) == small


def test_default_tile_for_wide_digits_is_accepted():
    """11-bit digits with the tile left at its default resolve to a 512-thread tile (workspace
    sizing goes through the same resolution, so a size comes back instead of an error)."""
    assert _abi.sa_sort_ws_bytes(1000, _abi.Tuning(digit_bits=11)) > 0
    assert _abi.sa_sort_ws_bytes(1000, _abi.Tuning(digit_bits=8)) > 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "_LIB", str(tmp_path / "libsaasm.so"))
    with pytest.raises(ImportError):
        _abi.load()


def test_one_hip_runtime_whatever_the_import_order():
    """Loading the library before anything imports torch still leaves one HIP runtime and one
    HSA runtime mapped in the process once torch is in use (a fresh interpreter, no GPU needed:
    the mapped files are read from /proc/self/maps)."""
    import subprocess
    import sys
    code = ("from paper_1404_3456_amd import _abi\n"
            "_abi.load()\n"
            "import torch\n"
            "torch.zeros(1)\n"
            "libs = set()\n"
            "for line in open('/proc/self/maps'):\n"
            "    f = line.split()[-1]\n"
            "    if 'libamdhip64' in f or 'libhsa-runtime64' in f:\n"
            "        libs.add(os.path.realpath(f))\n"
            "print(len([f for f in libs if 'amdhip' in f]), len([f for f in libs if 'hsa' in f]))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", "import os\n" + code], cwd=root,
                         capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.split()[-2:] == ["1", "1"], out.stdout


def test_one_workspace_covers_the_path():
    """sa_workspace_bytes is at least what each call of the path asks for: sa_build (default
    tuning), sa_lcp (both LCP forms) and sa_overlaps with up to n candidate matches."""
    for n, m in ((1, 1), (100, 3), (80_400, 400), (50_100_000, 100_000), ((1 << 31) - 3, 2_147_484)):
        w = _abi.sa_workspace_bytes(n, m)
        assert w >= _abi.sa_build_ws_bytes(n), n
        assert w >= _abi.sa_lcp_ws_bytes(n), n
        assert w >= _abi.sa_overlaps_ws_bytes(n, m, n), n
        assert w >= _abi.sa_overlaps_ws_bytes(n, m, 0), n
        assert _abi.sa_workspace_bytes(n, 0) >= w  # no read bound: as if every byte were a read
    assert _abi.sa_workspace_bytes(0, 0) == -1


def test_lcp_status_and_batched_lcp_host_checks():
    lib = _abi.load()
    dummy = ctypes.c_void_p(16)
    assert lib.sa_lcp_status(None, None) == _abi.SA_ERR_INVALID
    off = np.array([0, 50, 100], dtype=np.int64)
    P = ctypes.c_void_p
    # NULL text; then a workspace too small; the LCP output pointer is optional
    assert lib.sa_build_batched(None, 100, off.ctypes.data_as(P), 2, dummy, None, None, dummy,
                                1 << 20, None, 0, None, None) == _abi.SA_ERR_INVALID
    assert lib.sa_build_batched(dummy, 100, off.ctypes.data_as(P), 2, dummy, None, dummy, dummy,
                                16, None, 0, None, None) == _abi.SA_ERR_NOMEM
    # the batched workspace holds the LCP's room as well
    assert _abi.sa_build_batched_ws_bytes(1_000_000, 2) > _abi.sa_build_ws_bytes(1_000_000)
