"""Oracle for C = A*B on CSR inputs -- TEST INFRASTRUCTURE.

A plain CPU implementation of the paper's row-by-row sparse product (Section
III-A, Algorithm 1): see ``spgemm_oracle.c`` for what it computes and for the
readings taken where the paper is silent.  It exists to check the GPU library.
Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import it; the GPU library and its Python binding never do, and this
package imports nothing from them.

Inputs are :class:`synth.CSR`-like objects (``rows``, ``cols``, ``row_ptr``,
``col``, ``val``).  Values are promoted to float64 before the call (exact for
float32), indices to int64 row pointers / int32 columns.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spgemm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with the host C compiler (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def load_library(path: str):
    """Open a compiled oracle library and declare its entry points."""
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.oracle_spgemm_count.argtypes = [i64, P, P, P, P, P, i64, P, P, ctypes.c_int]
    lib.oracle_spgemm_count.restype = ctypes.c_int
    lib.oracle_spgemm_fill.argtypes = [i64, P, P, P, P, P, P, P, i64, P, P, P, P, ctypes.c_int]
    lib.oracle_spgemm_fill.restype = ctypes.c_int
    lib.oracle_max_threads.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = load_library(_LIB)
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


@dataclass
class OracleResult:
    """Rows ``rows`` of C: CSR over those rows (int64 row_ptr), plus the
    per-entry scale S_ij = sum |a_ik b_kj| and per-row product counts."""

    rows: np.ndarray        # which rows of C (int64)
    n_cols: int
    row_ptr: np.ndarray     # int64, len(rows)+1
    col: np.ndarray         # int32
    val: np.ndarray         # float64
    sabs: np.ndarray        # float64
    products: np.ndarray    # int64 per listed row

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def total_products(self) -> int:
        return int(self.products.sum())


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(A, B):
    if A.cols != B.rows:
        raise ValueError("inner dimensions differ: A is %dx%d, B is %dx%d" % (A.rows, A.cols, B.rows, B.cols))
    for M, name in ((A, "A"), (B, "B")):
        rp = np.asarray(M.row_ptr, dtype=np.int64)
        if rp.shape != (M.rows + 1,) or rp[0] != 0 or np.any(np.diff(rp) < 0):
            raise ValueError("%s: bad row_ptr" % name)
        if len(M.col) < rp[-1] or len(M.val) < rp[-1]:
            raise ValueError("%s: arrays shorter than row_ptr[-1]" % name)
        c = np.asarray(M.col[: rp[-1]])
        if c.size and (c.min() < 0 or c.max() >= M.cols):
            raise ValueError("%s: column index out of range" % name)


def spgemm(A, B, rows=None, threads: int = 1, with_values: bool = True, lib=None) -> OracleResult:
    """C = A*B restricted to ``rows`` (default: all rows of A).

    With ``with_values=False`` only the pattern pass runs: ``row_ptr`` and
    ``products`` are filled, ``col``/``val``/``sabs`` are left zero.  ``lib``
    selects another compiled oracle library (default: this package's)."""
    _check(A, B)
    lib = _load() if lib is None else lib
    a_rp = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
    b_rp = np.ascontiguousarray(B.row_ptr, dtype=np.int64)
    a_col = np.ascontiguousarray(A.col, dtype=np.int32)
    b_col = np.ascontiguousarray(B.col, dtype=np.int32)
    if rows is None:
        rows = np.arange(A.rows, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= A.rows):
        raise ValueError("row index out of range")
    nr = rows.size
    nnz = np.zeros(nr, dtype=np.int64)
    prod = np.zeros(nr, dtype=np.int64)
    rc = lib.oracle_spgemm_count(int(B.cols), _p(a_rp), _p(a_col), _p(b_rp), _p(b_col), _p(rows),
                                 nr, _p(nnz), _p(prod), int(threads))
    if rc != 0:
        raise MemoryError("oracle pattern pass failed")
    rp = np.zeros(nr + 1, dtype=np.int64)
    np.cumsum(nnz, out=rp[1:])
    total = int(rp[-1])
    col = np.zeros(total, dtype=np.int32)
    val = np.zeros(total, dtype=np.float64)
    sabs = np.zeros(total, dtype=np.float64)
    if with_values:
        a_val = np.ascontiguousarray(A.val, dtype=np.float64)
        b_val = np.ascontiguousarray(B.val, dtype=np.float64)
        rc = lib.oracle_spgemm_fill(int(B.cols), _p(a_rp), _p(a_col), _p(a_val), _p(b_rp), _p(b_col),
                                    _p(b_val), _p(rows), nr, _p(rp), _p(col), _p(val), _p(sabs),
                                    int(threads))
        if rc != 0:
            raise MemoryError("oracle value pass failed")
    return OracleResult(rows, int(B.cols), rp, col, val, sabs, prod)


def row_products(A, B) -> np.ndarray:
    """Per-row partial-product counts of A*B (pattern pass only)."""
    return spgemm(A, B, with_values=False).products
