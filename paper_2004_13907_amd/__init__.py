"""Sparse general matrix-matrix product C = A*B on CSR operands for AMD
Instinct MI355X (gfx950): the row-by-row product of the REAP paper (Section
III-A, Algorithm 1) as hand-written HIP kernels behind a C ABI.

The functions named like the C entry points (``reap_spgemm_create``,
``reap_spgemm_symbolic``, ``reap_spgemm_numeric``, ``reap_spgemm_destroy``)
only marshal arguments; PyTorch supplies device memory and the stream.
``spgemm(A, B)`` chains them.  The HIP library must be built; there is no CPU
path.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _capi
from ._capi import (REAP_ERR_INDEX_OVERFLOW, REAP_F32, REAP_F64, REAP_I32, REAP_I64, REAP_OK,
                    reap_bin_stats_t, reap_csr_t, reap_options_t)

__all__ = [
    "DeviceCSR",
    "SpGEMMError",
    "Plan",
    "Batch",
    "spgemm",
    "spgemm_batch",
    "reap_spgemm_create",
    "reap_spgemm_symbolic",
    "reap_spgemm_symbolic_noalloc",
    "reap_spgemm_numeric",
    "reap_spgemm_batch_symbolic",
    "reap_spgemm_batch_numeric",
    "reap_spgemm_workspace_query",
    "reap_csr_transpose",
    "transpose",
    "reap_spgemm_destroy",
    "reap_spgemm_bin_stats",
    "reap_spgemm_phase_times",
    "reap_spgemm_phase_reset",
    "reap_status_string",
    "library_path",
]


class SpGEMMError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = int(status)
        msg = reap_status_string(status)
        super().__init__("%s: %s (status %d)" % (where or "reap_spgemm", msg, self.status))


def library_path() -> str:
    return _capi.LIB_PATH


def reap_status_string(status: int) -> str:
    return _capi.load().reap_status_string(int(status)).decode()


def _dtype_code(dtype) -> int:
    if dtype == torch.float64:
        return REAP_F64
    if dtype == torch.float32:
        return REAP_F32
    raise TypeError("values must be float32 or float64, got %s" % dtype)


def _index_code(dtype) -> int:
    if dtype == torch.int32:
        return REAP_I32
    if dtype == torch.int64:
        return REAP_I64
    raise TypeError("row pointers must be int32 or int64, got %s" % dtype)


@dataclass
class DeviceCSR:
    """CSR operand held in torch device tensors."""

    rows: int
    cols: int
    row_ptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @property
    def dtype(self):
        return self.val.dtype

    @classmethod
    def from_host(cls, M, device="cuda", dtype=None, index_dtype=None) -> "DeviceCSR":
        """From any object with rows, cols, row_ptr, col, val (numpy arrays)."""
        rp = np.asarray(M.row_ptr)
        if index_dtype is not None:
            rp = rp.astype(np.int64 if index_dtype == torch.int64 else np.int32)
        val = np.asarray(M.val)
        if dtype is not None:
            val = val.astype(np.float64 if dtype == torch.float64 else np.float32)
        nnz = int(rp[-1]) if rp.size else 0
        return cls(int(M.rows), int(M.cols),
                   torch.from_numpy(np.ascontiguousarray(rp)).to(device),
                   torch.from_numpy(np.ascontiguousarray(np.asarray(M.col)[:nnz], dtype=np.int32)).to(device),
                   torch.from_numpy(np.ascontiguousarray(val[:nnz])).to(device))

    def to_host(self):
        return (self.row_ptr.cpu().numpy(), self.col.cpu().numpy(), self.val.cpu().numpy())

    def c_struct(self) -> reap_csr_t:
        # built once per set of tensors (the same operand is passed call after call)
        key = (id(self.row_ptr), id(self.col), id(self.val), self.rows, self.cols)
        cached = self.__dict__.get("_cs")
        if cached is not None and cached[0] == key:
            return cached[1]
        s = self._make_struct()
        self.__dict__["_cs"] = (key, s)
        return s

    def _make_struct(self) -> reap_csr_t:
        for t in (self.row_ptr, self.col, self.val):
            if not t.is_contiguous():
                raise ValueError("CSR tensors must be contiguous")
        if self.col.dtype != torch.int32:
            raise TypeError("column indices must be int32")
        s = reap_csr_t()
        s.rows = self.rows
        s.cols = self.cols
        s.nnz = self.nnz
        s.row_ptr_type = _index_code(self.row_ptr.dtype)
        s.row_ptr = self.row_ptr.data_ptr()
        s.col_idx = self.col.data_ptr() if self.nnz else None
        s.values = self.val.data_ptr() if self.nnz else None
        return s


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _options(**kw) -> reap_options_t:
    o = reap_options_t()
    for k, v in kw.items():
        if not hasattr(o, k) or k == "reserved":
            raise TypeError("unknown option %r" % k)
        setattr(o, k, int(v))
    return o


# --- thin wrappers, same names as the C entry points -------------------------

def reap_spgemm_create(dtype, c_index_dtype=torch.int32, stream=None, **options) -> ctypes.c_void_p:
    lib = _capi.load()
    h = ctypes.c_void_p()
    o = _options(**options)
    st = lib.reap_spgemm_create(ctypes.byref(h), _dtype_code(dtype), _index_code(c_index_dtype),
                                ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(o))
    if st != REAP_OK:
        raise SpGEMMError(st, "reap_spgemm_create")
    return h


def reap_spgemm_symbolic(plan, A: DeviceCSR, B: DeviceCSR, c_row_ptr: torch.Tensor):
    """Returns (status, nnz(C), partial products, workspace bytes)."""
    lib = _capi.load()
    a, b = A.c_struct(), B.c_struct()
    nnz = ctypes.c_int64(0)
    prods = ctypes.c_int64(0)
    ws = ctypes.c_size_t(0)
    st = lib.reap_spgemm_symbolic(plan, ctypes.byref(a), ctypes.byref(b), ctypes.c_void_p(c_row_ptr.data_ptr()),
                                  ctypes.byref(nnz), ctypes.byref(prods), ctypes.byref(ws))
    return st, int(nnz.value), int(prods.value), int(ws.value)


def reap_spgemm_symbolic_noalloc(plan, A: DeviceCSR, B: DeviceCSR, c_row_ptr: torch.Tensor):
    """The allocation-free symbolic pass; returns (status, nnz(C), partial products)."""
    lib = _capi.load()
    a, b = A.c_struct(), B.c_struct()
    nnz = ctypes.c_int64(0)
    prods = ctypes.c_int64(0)
    st = lib.reap_spgemm_symbolic_noalloc(plan, ctypes.byref(a), ctypes.byref(b),
                                          ctypes.c_void_p(c_row_ptr.data_ptr()), ctypes.byref(nnz),
                                          ctypes.byref(prods))
    return st, int(nnz.value), int(prods.value)


def reap_spgemm_numeric(plan, A: DeviceCSR, B: DeviceCSR, c_row_ptr: torch.Tensor, c_col: torch.Tensor,
                        c_val: torch.Tensor) -> int:
    lib = _capi.load()
    a, b = A.c_struct(), B.c_struct()
    return lib.reap_spgemm_numeric(plan, ctypes.byref(a), ctypes.byref(b),
                                   ctypes.c_void_p(c_row_ptr.data_ptr()),
                                   ctypes.c_void_p(c_col.data_ptr() if c_col.numel() else None),
                                   ctypes.c_void_p(c_val.data_ptr() if c_val.numel() else None))


def reap_spgemm_batch_symbolic(plan, As, Bs, c_row_ptrs):
    """Returns (status, [nnz(C_q)], [partial products of q], workspace bytes)."""
    lib = _capi.load()
    n = len(As)
    if len(Bs) != n or len(c_row_ptrs) != n:
        raise ValueError("A, B and C row-pointer lists differ in length")
    a = (reap_csr_t * n)(*[x.c_struct() for x in As])
    b = (reap_csr_t * n)(*[x.c_struct() for x in Bs])
    rp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in c_row_ptrs])
    nnz = (ctypes.c_int64 * n)()
    prods = (ctypes.c_int64 * n)()
    ws = ctypes.c_size_t(0)
    st = lib.reap_spgemm_batch_symbolic(plan, n, a, b, rp, nnz, prods, ctypes.byref(ws))
    return st, [int(x) for x in nnz], [int(x) for x in prods], int(ws.value)


def reap_spgemm_batch_numeric(plan, As, Bs, c_row_ptrs, c_cols, c_vals) -> int:
    lib = _capi.load()
    n = len(As)
    a = (reap_csr_t * n)(*[x.c_struct() for x in As])
    b = (reap_csr_t * n)(*[x.c_struct() for x in Bs])
    rp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in c_row_ptrs])
    cc = (ctypes.c_void_p * n)(*[(t.data_ptr() if t.numel() else None) for t in c_cols])
    cv = (ctypes.c_void_p * n)(*[(t.data_ptr() if t.numel() else None) for t in c_vals])
    return lib.reap_spgemm_batch_numeric(plan, n, a, b, rp, cc, cv)


def reap_spgemm_workspace_query(plan, As, Bs) -> int:
    """Device bytes the plan will hold after a (batched) symbolic call on
    these operands (raises on an invalid batch)."""
    n = len(As)
    if len(Bs) != n:
        raise ValueError("A and B lists differ in length")
    a = (reap_csr_t * n)(*[x.c_struct() for x in As])
    b = (reap_csr_t * n)(*[x.c_struct() for x in Bs])
    out = ctypes.c_size_t(0)
    st = _capi.load().reap_spgemm_workspace_query(plan, n, a, b, ctypes.byref(out))
    if st != REAP_OK:
        raise SpGEMMError(st, "reap_spgemm_workspace_query")
    return int(out.value)


def reap_csr_transpose(plan, A: DeviceCSR, t_row_ptr: torch.Tensor, t_col: torch.Tensor, t_val: torch.Tensor) -> int:
    lib = _capi.load()
    a = A.c_struct()
    return lib.reap_csr_transpose(plan, ctypes.byref(a), ctypes.c_void_p(t_row_ptr.data_ptr()),
                                  ctypes.c_void_p(t_col.data_ptr() if t_col.numel() else None),
                                  ctypes.c_void_p(t_val.data_ptr() if t_val.numel() else None))


def reap_spgemm_destroy(plan) -> int:
    return _capi.load().reap_spgemm_destroy(plan)


def reap_spgemm_bin_stats(plan) -> dict:
    s = reap_bin_stats_t()
    st = _capi.load().reap_spgemm_bin_stats(plan, ctypes.byref(s))
    if st != REAP_OK:
        raise SpGEMMError(st, "reap_spgemm_bin_stats")
    return {f: int(getattr(s, f)) for f, _ in reap_bin_stats_t._fields_}


def reap_spgemm_phase_times(plan) -> dict:
    out = (ctypes.c_float * 8)()
    st = _capi.load().reap_spgemm_phase_times(plan, out, 8)
    if st != REAP_OK:
        raise SpGEMMError(st, "reap_spgemm_phase_times")
    names = ("symbolic", "scan", "numeric_wave_bitmap", "numeric_wave_hash", "numeric_group", "numeric")
    d = {n: float(out[i]) for i, n in enumerate(names)}
    d["calls"] = int(out[7])
    return d


def reap_spgemm_phase_reset(plan) -> None:
    st = _capi.load().reap_spgemm_phase_reset(plan)
    if st != REAP_OK:
        raise SpGEMMError(st, "reap_spgemm_phase_reset")


# --- convenience ---------------------------------------------------------------

class Plan:
    """A product plan bound to one dtype, C row-pointer type and stream."""

    def __init__(self, dtype=torch.float64, c_index_dtype=torch.int32, stream=None, **options):
        self.dtype = dtype
        self.c_index_dtype = c_index_dtype
        self.stream = stream
        self.options = options
        self.handle = reap_spgemm_create(dtype, c_index_dtype, stream, **options)
        self.last_products = None
        self.last_nnz = None
        self.workspace_bytes = 0

    def _check_dtypes(self, A: DeviceCSR, B: DeviceCSR):
        if A.val.dtype != self.dtype or B.val.dtype != self.dtype:
            raise TypeError("operand values are %s/%s, the plan computes in %s" % (A.val.dtype, B.val.dtype,
                                                                                  self.dtype))

    def symbolic(self, A: DeviceCSR, B: DeviceCSR, c_row_ptr: torch.Tensor | None = None):
        self._check_dtypes(A, B)
        if c_row_ptr is None:
            c_row_ptr = torch.empty(A.rows + 1, dtype=self.c_index_dtype, device=A.row_ptr.device)
        st, nnz, prods, ws = reap_spgemm_symbolic(self.handle, A, B, c_row_ptr)
        if st != REAP_OK:
            raise SpGEMMError(st, "reap_spgemm_symbolic")
        self.last_nnz, self.last_products, self.workspace_bytes = nnz, prods, ws
        return c_row_ptr, nnz, prods

    def numeric(self, A: DeviceCSR, B: DeviceCSR, c_row_ptr: torch.Tensor, c_col=None, c_val=None):
        self._check_dtypes(A, B)
        nnz = self.last_nnz if self.last_nnz is not None else 0
        dev = A.row_ptr.device
        if c_col is None:
            c_col = torch.empty(nnz, dtype=torch.int32, device=dev)
        if c_val is None:
            c_val = torch.empty(nnz, dtype=self.dtype, device=dev)
        st = reap_spgemm_numeric(self.handle, A, B, c_row_ptr, c_col, c_val)
        if st != REAP_OK:
            raise SpGEMMError(st, "reap_spgemm_numeric")
        return c_col, c_val

    def bin_stats(self) -> dict:
        return reap_spgemm_bin_stats(self.handle)

    def phase_times(self) -> dict:
        return reap_spgemm_phase_times(self.handle)

    def phase_reset(self) -> None:
        reap_spgemm_phase_reset(self.handle)

    def close(self):
        if self.handle is not None:
            reap_spgemm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Independent products C_q = A_q * B_q computed together: one launch per
    kernel for the whole batch, or, with ``graph=True``, one HIP graph launch
    per pass, captured on first use and replayed while the batch's launch
    shape repeats.  C's row pointers, columns and values live in three device
    buffers; the results are views into them.  Work runs on ``stream`` (a
    fresh torch stream when ``graph`` is set and none is given)."""

    def __init__(self, dtype=torch.float64, c_index_dtype=torch.int32, stream=None, graph: bool = False,
                 **options):
        if graph and stream is None:
            stream = torch.cuda.Stream()
        self.stream = stream
        self.dtype = dtype
        self.c_index_dtype = c_index_dtype
        self.plan = Plan(dtype, c_index_dtype, stream=stream, graph=int(bool(graph)), **options)
        self.nnz = []
        self.products = []
        self.workspace_bytes = 0
        self._rp = None
        self._rp_views = []

    def _ctx(self):
        return torch.cuda.stream(self.stream) if self.stream is not None else _NullCtx()

    def workspace_query(self, As, Bs) -> int:
        """Device bytes the batch's plan will hold once symbolic(As, Bs) has
        returned (host-only; nothing is allocated)."""
        return reap_spgemm_workspace_query(self.plan.handle, As, Bs)

    def symbolic(self, As, Bs, fresh: bool = False):
        """Per-product nnz(C_q); row pointers are written on the device, into
        a buffer the batch reuses call after call, or (``fresh=True``) into a
        new one that results of later calls do not overwrite."""
        if len(As) != len(Bs) or not As:
            raise ValueError("need equally many (and at least one) A and B operands")
        for A, B in zip(As, Bs):
            self.plan._check_dtypes(A, B)
        total = sum(A.rows + 1 for A in As)
        dev = As[0].row_ptr.device
        with self._ctx():
            if fresh or self._rp is None or self._rp.numel() < total or self._rp.dtype != self.c_index_dtype:
                self._rp = torch.empty(total, dtype=self.c_index_dtype, device=dev)
        views, o = [], 0
        for A in As:
            views.append(self._rp[o:o + A.rows + 1])
            o += A.rows + 1
        st, nnz, prods, ws = reap_spgemm_batch_symbolic(self.plan.handle, As, Bs, views)
        if st != REAP_OK:
            raise SpGEMMError(st, "reap_spgemm_batch_symbolic")
        self._rp_views = views
        self.nnz, self.products, self.workspace_bytes = nnz, prods, ws
        return nnz

    def numeric(self, As, Bs, out=None):
        """Writes every C_q; returns the list of DeviceCSR results (views into
        the batch's buffers, or into ``out`` = (col, val) buffers of at least
        sum(nnz) elements).  Asynchronous on the batch's stream."""
        total = sum(self.nnz)
        dev = As[0].row_ptr.device
        with self._ctx():
            if out is None:
                col = torch.empty(max(total, 1), dtype=torch.int32, device=dev)
                val = torch.empty(max(total, 1), dtype=self.dtype, device=dev)
            else:
                col, val = out
        cols, vals, o = [], [], 0
        for z in self.nnz:
            cols.append(col[o:o + z])
            vals.append(val[o:o + z])
            o += z
        st = reap_spgemm_batch_numeric(self.plan.handle, As, Bs, self._rp_views, cols, vals)
        if st != REAP_OK:
            raise SpGEMMError(st, "reap_spgemm_batch_numeric")
        return [DeviceCSR(A.rows, B.cols, rp, c, v) for A, B, rp, c, v in zip(As, Bs, self._rp_views, cols, vals)]

    def synchronize(self):
        if self.stream is not None:
            self.stream.synchronize()
        else:
            torch.cuda.synchronize()

    def close(self):
        self.plan.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class _NullCtx:
    def __enter__(self):
        return self

    def __exit__(self, *exc):
        return False


def spgemm_batch(As, Bs, dtype=None, c_index_dtype=torch.int32, graph: bool = False, **options):
    """C_q = A_q * B_q for every q, in one batch; returns the list of results."""
    dtype = dtype or As[0].dtype
    with Batch(dtype, c_index_dtype, graph=graph, **options) as b:
        b.symbolic(As, Bs)
        out = b.numeric(As, Bs)
        b.synchronize()
    return out


def transpose(A: DeviceCSR, plan: Plan | None = None) -> DeviceCSR:
    """A^T on the device (row pointers of A's index type).  Asynchronous on the
    plan's stream (torch's current stream for a temporary plan, which is
    synchronised before it is released)."""
    own = plan is None
    if own:
        plan = Plan(A.dtype, torch.int32)
    try:
        dev = A.row_ptr.device
        rp = torch.empty(A.cols + 1, dtype=A.row_ptr.dtype, device=dev)
        col = torch.empty(A.nnz, dtype=torch.int32, device=dev)
        val = torch.empty(A.nnz, dtype=A.dtype, device=dev)
        st = reap_csr_transpose(plan.handle, A, rp, col, val)
        if st != REAP_OK:
            raise SpGEMMError(st, "reap_csr_transpose")
        return DeviceCSR(A.cols, A.rows, rp, col, val)
    finally:
        if own:
            plan.close()


def spgemm(A: DeviceCSR, B: DeviceCSR, c_index_dtype=None, plan: Plan | None = None, **options) -> DeviceCSR:
    """C = A*B.  With ``c_index_dtype=None`` the row pointer is int32 and is
    widened to int64 only when nnz(C) does not fit."""
    own = plan is None
    if own:
        plan = Plan(A.dtype, c_index_dtype or torch.int32, **options)
    try:
        try:
            rp, nnz, _ = plan.symbolic(A, B)
        except SpGEMMError as e:
            if e.status != REAP_ERR_INDEX_OVERFLOW or c_index_dtype is not None or not own:
                raise
            plan.close()
            plan = Plan(A.dtype, torch.int64, **options)
            rp, nnz, _ = plan.symbolic(A, B)
        col, val = plan.numeric(A, B, rp)
        return DeviceCSR(A.rows, B.cols, rp, col, val)
    finally:
        if own:
            plan.close()
