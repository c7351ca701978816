"""ctypes declarations of the C ABI in include/reap_spgemm.h (argument
marshalling only; every step of the product runs in the HIP library)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libreap_spgemm.so")

REAP_OK = 0
REAP_ERR_INVALID_ARG = 1
REAP_ERR_BAD_CSR = 2
REAP_ERR_INDEX_OVERFLOW = 3
REAP_ERR_OUT_OF_MEMORY = 4
REAP_ERR_STATE = 5
REAP_ERR_HIP = 6
REAP_ERR_TOO_LARGE = 7
REAP_NOALLOC_SCRATCH_BYTES = 64 << 20

REAP_F32 = 0
REAP_F64 = 1
REAP_I32 = 0
REAP_I64 = 1

# Every function the header declares; the CPU tests check the library exports them.
EXPORTED = (
    "reap_spgemm_create",
    "reap_spgemm_symbolic",
    "reap_spgemm_symbolic_noalloc",
    "reap_spgemm_numeric",
    "reap_spgemm_batch_symbolic",
    "reap_spgemm_batch_numeric",
    "reap_spgemm_workspace_query",
    "reap_csr_transpose",
    "reap_spgemm_destroy",
    "reap_spgemm_bin_stats",
    "reap_spgemm_phase_times",
    "reap_spgemm_phase_reset",
    "reap_status_string",
    "reap_version",
)


class reap_csr_t(ctypes.Structure):
    _fields_ = [
        ("rows", ctypes.c_int64),
        ("cols", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("row_ptr_type", ctypes.c_int),
        ("row_ptr", ctypes.c_void_p),
        ("col_idx", ctypes.c_void_p),
        ("values", ctypes.c_void_p),
    ]


class reap_options_t(ctypes.Structure):
    _fields_ = [
        ("validate", ctypes.c_int32),
        ("wave_max_products", ctypes.c_int32),
        ("wave_max_span", ctypes.c_int32),
        ("wave_hash_products", ctypes.c_int32),
        ("group_lds_span", ctypes.c_int32),
        ("group_lds_values", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("wave_small_values", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("long_workgroups_per_cu", ctypes.c_int32),
        ("test_fail_alloc", ctypes.c_int32),
        ("scan_onepass_tiles", ctypes.c_int32),
        ("mid_values", ctypes.c_int32),
        ("long_sym_narrow", ctypes.c_int32),
        ("wave_hash_slots", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 1),
    ]


class reap_bin_stats_t(ctypes.Structure):
    _fields_ = [
        ("empty", ctypes.c_int64),
        ("wave_bitmap", ctypes.c_int64),
        ("wave_hash", ctypes.c_int64),
        ("group", ctypes.c_int64),
        ("max_row_products", ctypes.c_int64),
        ("max_row_nnz", ctypes.c_int64),
        ("long_segments_lds", ctypes.c_int64),
        ("long_segments_chunked", ctypes.c_int64),
        ("long_segments_device", ctypes.c_int64),
        ("group_medium", ctypes.c_int64),
    ]


_lib = None


def load():
    """Open the HIP library; raises if it has not been built (there is no
    fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libreap_spgemm.so is not built (run paper_2004_13907_amd.build.build() "
                           "or __graft_entry__.build()); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    st = ctypes.c_int
    lib.reap_spgemm_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, ctypes.c_int, P,
                                       ctypes.POINTER(reap_options_t)]
    lib.reap_spgemm_create.restype = st
    lib.reap_spgemm_symbolic.argtypes = [P, ctypes.POINTER(reap_csr_t), ctypes.POINTER(reap_csr_t), P,
                                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_size_t)]
    lib.reap_spgemm_symbolic.restype = st
    lib.reap_spgemm_symbolic_noalloc.argtypes = [P, ctypes.POINTER(reap_csr_t), ctypes.POINTER(reap_csr_t), P,
                                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.reap_spgemm_symbolic_noalloc.restype = st
    lib.reap_spgemm_numeric.argtypes = [P, ctypes.POINTER(reap_csr_t), ctypes.POINTER(reap_csr_t), P, P, P]
    lib.reap_spgemm_numeric.restype = st
    PP = ctypes.POINTER(P)
    lib.reap_spgemm_batch_symbolic.argtypes = [P, ctypes.c_int64, ctypes.POINTER(reap_csr_t),
                                               ctypes.POINTER(reap_csr_t), PP, ctypes.POINTER(ctypes.c_int64),
                                               ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_size_t)]
    lib.reap_spgemm_batch_symbolic.restype = st
    lib.reap_spgemm_batch_numeric.argtypes = [P, ctypes.c_int64, ctypes.POINTER(reap_csr_t),
                                              ctypes.POINTER(reap_csr_t), PP, PP, PP]
    lib.reap_spgemm_batch_numeric.restype = st
    lib.reap_spgemm_workspace_query.argtypes = [P, ctypes.c_int64, ctypes.POINTER(reap_csr_t),
                                                ctypes.POINTER(reap_csr_t), ctypes.POINTER(ctypes.c_size_t)]
    lib.reap_spgemm_workspace_query.restype = st
    lib.reap_csr_transpose.argtypes = [P, ctypes.POINTER(reap_csr_t), P, P, P]
    lib.reap_csr_transpose.restype = st
    lib.reap_spgemm_destroy.argtypes = [P]
    lib.reap_spgemm_destroy.restype = st
    lib.reap_spgemm_bin_stats.argtypes = [P, ctypes.POINTER(reap_bin_stats_t)]
    lib.reap_spgemm_bin_stats.restype = st
    lib.reap_spgemm_phase_times.argtypes = [P, ctypes.POINTER(ctypes.c_float), ctypes.c_int]
    lib.reap_spgemm_phase_times.restype = st
    lib.reap_spgemm_phase_reset.argtypes = [P]
    lib.reap_spgemm_phase_reset.restype = st
    lib.reap_status_string.argtypes = [ctypes.c_int]
    lib.reap_status_string.restype = ctypes.c_char_p
    lib.reap_version.argtypes = []
    lib.reap_version.restype = ctypes.c_char_p
    _lib = lib
    return lib
