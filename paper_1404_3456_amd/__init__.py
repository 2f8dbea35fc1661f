"""MI355X suffix-array / read-overlap library: Python binding over the C ABI in
include/saasm.h.

Argument marshalling only: every step runs in the HIP kernels of libsaasm.so.  PyTorch supplies
device memory (the outputs and the scratch workspace) and the stream.  Importing the package
does not load the library; the first call does, and raises if libsaasm.so is missing.
"""
from __future__ import annotations

from ._abi import (  # noqa: F401
    AsmServer,
    SaasmError,
    SA_PENDING,
    SA_OK,
    SA_ERR_ALPHABET,
    SA_ERR_CAPACITY,
    SA_ERR_HIP,
    SA_ERR_INVALID,
    SA_ERR_NOMEM,
    SA_ERR_NOTFOUND,
    SA_ERR_TOO_LARGE,
    Tuning,
    lib_path,
    load,
    sa_build,
    sa_build_batched,
    sa_build_batched_ws_bytes,
    sa_build_dc3,
    sa_build_dc3_ws_bytes,
    sa_build_ws_bytes,
    sa_copy_u32,
    sa_lcp,
    sa_lcp_status,
    sa_lcp_plcp_min,
    sa_lcp_set_chunk,
    sa_lcp_ws_bytes,
    sa_lookup,
    sa_lookup_ws_bytes,
    sa_overlap_path,
    sa_reconstruct,
    sa_reconstruct_host,
    sa_revcomp_text,
    sa_strand_rows,
    sa_overlaps_rc,
    sa_overlaps,
    sa_overlaps_ws_bytes,
    sa_pack,
    sa_path,
    sa_sort_pairs,
    sa_sort_ws_bytes,
    sa_timing_enable,
    sa_timing_get,
    sa_timing_items,
    sa_timing_reset,
    sa_version,
    sa_last_error,
    sa_workspace_bytes,
)
