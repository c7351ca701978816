"""Comparison of the GPU library's output with the oracle.

Pattern (row pointer and column indices) must match bit for bit.  Values are
compared per entry against the FP64 oracle with the error normalised by the
entry's scale S_ij = sum_k |a_ik b_kj|:

    |c_gpu - c_oracle| <= tol * S_ij,   tol = 1e-12 (FP64), 1e-5 (FP32),

which is the plain relative error wherever the products do not cancel
(S_ij = |c_ij|).  Where S_ij = 0 the GPU value must be exactly 0.
"""
from __future__ import annotations

import numpy as np

TOL = {np.dtype(np.float64): 1e-12, np.dtype(np.float32): 1e-5}


def tolerance(dtype) -> float:
    return TOL[np.dtype(dtype)]


def compare_rows(ref, rows, gpu_rp, gpu_col, gpu_val, dtype, label=""):
    """Compare GPU rows ``rows`` (numpy index array) with the oracle result
    ``ref`` (computed for exactly those rows, in that order).  ``gpu_rp`` is
    the full row pointer of C; ``gpu_col``/``gpu_val`` the full arrays."""
    tol = tolerance(dtype)
    rows = np.asarray(rows, dtype=np.int64)
    gpu_rp = np.asarray(gpu_rp, dtype=np.int64)
    lens = gpu_rp[rows + 1] - gpu_rp[rows]
    ref_lens = np.diff(ref.row_ptr)
    bad = np.nonzero(lens != ref_lens)[0]
    assert bad.size == 0, "%s: row lengths differ at rows %s (gpu %s, oracle %s)" % (
        label, rows[bad[:5]], lens[bad[:5]], ref_lens[bad[:5]])
    if rows.size == 0:
        return {"max_err": 0.0, "entries": 0}
    idx = np.concatenate([np.arange(gpu_rp[i], gpu_rp[i + 1]) for i in rows]) if lens.sum() else np.zeros(0, np.int64)
    gc = np.asarray(gpu_col)[idx]
    gv = np.asarray(gpu_val)[idx].astype(np.float64)
    if not np.array_equal(gc, ref.col):
        k = int(np.nonzero(gc != ref.col)[0][0])
        raise AssertionError("%s: column mismatch at entry %d: gpu %d, oracle %d" % (label, k, gc[k], ref.col[k]))
    err = np.abs(gv - ref.val)
    scale = ref.sabs
    zero = scale == 0
    assert np.all(gv[zero] == 0.0), "%s: nonzero value where every product is zero" % label
    ratio = np.zeros_like(err)
    ratio[~zero] = err[~zero] / scale[~zero]
    worst = int(np.argmax(ratio)) if ratio.size else 0
    assert ratio.size == 0 or ratio[worst] <= tol, "%s: value error %.3e > %.1e at entry %d (gpu %r, oracle %r)" % (
        label, ratio[worst], tol, worst, gv[worst], ref.val[worst])
    rel = np.zeros_like(err)
    nz = ref.val != 0
    rel[nz] = err[nz] / np.abs(ref.val[nz])
    return {"max_err": float(ratio.max()) if ratio.size else 0.0,
            "max_plain_rel": float(rel.max()) if rel.size else 0.0,
            "over_tol_plain": int(np.sum(rel > tol)),
            "entries": int(idx.size)}


def compare_full(ref, gpu_rp, gpu_col, gpu_val, dtype, label=""):
    """Whole-matrix comparison: the oracle result covers every row."""
    gpu_rp = np.asarray(gpu_rp, dtype=np.int64)
    assert np.array_equal(gpu_rp, ref.row_ptr), "%s: row pointer differs" % label
    assert np.array_equal(np.asarray(gpu_col), ref.col), "%s: column indices differ" % label
    tol = tolerance(dtype)
    gv = np.asarray(gpu_val).astype(np.float64)
    err = np.abs(gv - ref.val)
    zero = ref.sabs == 0
    assert np.all(gv[zero] == 0.0), "%s: nonzero value where every product is zero" % label
    ratio = np.zeros_like(err)
    ratio[~zero] = err[~zero] / ref.sabs[~zero]
    if ratio.size:
        worst = int(np.argmax(ratio))
        assert ratio[worst] <= tol, "%s: value error %.3e > %.1e at entry %d (gpu %r, oracle %r)" % (
            label, ratio[worst], tol, worst, gv[worst], ref.val[worst])
    return {"max_err": float(ratio.max()) if ratio.size else 0.0, "entries": int(gv.size)}
