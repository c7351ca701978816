"""Independent pins for the oracle.

Each ``pin_*`` function checks the oracle (optionally a different compiled
build of it, ``lib``) against something that is not the oracle itself:
brute force in pure Python, integer arithmetic, closed forms of the 27-point
stencil, algebraic identities of the matrix product, or a third-party library
run as a comparator.  They raise ``AssertionError`` on a mismatch.  The same
functions serve the oracle tests and the planted-mistake tests, which require
every planted mistake to trip at least one pin.
"""
from __future__ import annotations

import math

import numpy as np

import oracle
import synth

U64 = 2.0 ** -53


def gamma(n: int) -> float:
    """Higham's gamma_n = n u / (1 - n u) for binary64 (u = 2^-53)."""
    nu = n * U64
    return nu / (1.0 - nu)


def brute_force(A, B):
    """Pure-Python product over dense structural indicators.

    Returns (pattern: set of (i, j), exact: dict (i, j) -> exactly rounded sum
    via math.fsum, terms: dict (i, j) -> number of products, absum)."""
    rpA = [int(x) for x in A.row_ptr]
    rpB = [int(x) for x in B.row_ptr]
    rows_b = []
    for k in range(B.rows):
        rows_b.append([(int(B.col[q]), float(B.val[q])) for q in range(rpB[k], rpB[k + 1])])
    pattern, terms = set(), {}
    prods = {}
    for i in range(A.rows):
        for p in range(rpA[i], rpA[i + 1]):
            k = int(A.col[p])
            a = float(A.val[p])
            for j, b in rows_b[k]:
                pattern.add((i, j))
                prods.setdefault((i, j), []).append(a * b)
    exact = {ij: math.fsum(v) for ij, v in prods.items()}
    absum = {ij: math.fsum(abs(x) for x in v) for ij, v in prods.items()}
    terms = {ij: len(v) for ij, v in prods.items()}
    return pattern, exact, terms, absum


def _entries(res):
    out = {}
    for r, i in enumerate(res.rows):
        for t in range(res.row_ptr[r], res.row_ptr[r + 1]):
            out[(int(i), int(res.col[t]))] = (float(res.val[t]), float(res.sabs[t]))
    return out


def pin_tiny_brute_force(lib=None, seeds=range(12)):
    """Pattern equals the structural product; values agree with the exactly
    rounded sum within gamma_n * sum|terms|; columns ascending per row."""
    for s in seeds:
        rng = np.random.default_rng(1000 + s)
        m, k, n = (int(x) for x in rng.integers(1, 24, size=3))
        A = synth.random_tiny(m, k, float(rng.uniform(0.05, 0.6)), seed=10 * s + 1,
                              allow_duplicates=bool(s % 3 == 0), unsorted=bool(s % 2),
                              empty_rows=0.2)
        B = synth.random_tiny(k, n, float(rng.uniform(0.05, 0.6)), seed=10 * s + 2,
                              allow_duplicates=bool(s % 4 == 1), unsorted=bool(s % 3 == 1),
                              empty_rows=0.2)
        res = oracle.spgemm(A, B, lib=lib)
        pattern, exact, terms, absum = brute_force(A, B)
        got = _entries(res)
        assert set(got) == pattern, "pattern differs from structural product (seed %d)" % s
        for r in range(len(res.rows)):
            cols = res.col[res.row_ptr[r]:res.row_ptr[r + 1]]
            assert np.all(np.diff(cols) > 0), "row columns not strictly ascending"
        for ij, (v, sa) in got.items():
            bound = gamma(terms[ij]) * absum[ij]
            assert abs(v - exact[ij]) <= bound, "value off at %s: %r vs %r" % (ij, v, exact[ij])
            assert abs(sa - absum[ij]) <= gamma(terms[ij]) * absum[ij], "scale off at %s" % (ij,)
        assert res.total_products == sum(terms.values())


def pin_dense_matmul(lib=None):
    """Against numpy's dense product of the summed-duplicate dense forms."""
    for s in range(6):
        A = synth.random_tiny(30, 25, 0.2, seed=500 + s, allow_duplicates=True)
        B = synth.random_tiny(25, 35, 0.2, seed=600 + s, unsorted=True)
        res = oracle.spgemm(A, B, lib=lib)
        D = synth.to_dense(A) @ synth.to_dense(B)
        got = np.zeros_like(D)
        for r in range(A.rows):
            for t in range(res.row_ptr[r], res.row_ptr[r + 1]):
                got[r, res.col[t]] = res.val[t]
        absA = np.abs(synth.to_dense(A))
        absB = np.abs(synth.to_dense(B))
        bound = gamma(2 * A.cols + 4) * (absA @ absB) * 2.0
        assert np.all(np.abs(got - D) <= bound + 1e-300)


def pin_integer_exact(lib=None):
    """Integer-valued inputs: every partial sum is an exact small integer, so
    values must equal the int64 product bit for bit (in any order)."""
    for s in range(5):
        A = synth.random_tiny(40, 33, 0.25, seed=700 + s, integer_values=True, allow_duplicates=True)
        B = synth.random_tiny(33, 37, 0.25, seed=800 + s, integer_values=True, unsorted=True)
        res = oracle.spgemm(A, B, lib=lib)
        DA = np.zeros((A.rows, A.cols), dtype=np.int64)
        np.add.at(DA, (np.repeat(np.arange(A.rows), np.diff(A.row_ptr)), A.col), A.val.astype(np.int64))
        DB = np.zeros((B.rows, B.cols), dtype=np.int64)
        np.add.at(DB, (np.repeat(np.arange(B.rows), np.diff(B.row_ptr)), B.col), B.val.astype(np.int64))
        IA = np.zeros_like(DA)
        IA[np.repeat(np.arange(A.rows), np.diff(A.row_ptr)), A.col] = 1
        IB = np.zeros_like(DB)
        IB[np.repeat(np.arange(B.rows), np.diff(B.row_ptr)), B.col] = 1
        P = (IA @ IB) > 0
        C = DA @ DB
        rows = np.repeat(np.arange(A.rows), np.diff(res.row_ptr))
        assert np.array_equal(np.nonzero(P)[0], rows) and np.array_equal(np.nonzero(P)[1], res.col)
        assert np.array_equal(res.val, C[P].astype(np.float64))


def _stencil_c2(x, g):
    return np.minimum(x, 2) + np.minimum(g - 1 - x, 2) + 1


def _overlap(xi, xj, g):
    lo = np.maximum(np.maximum(xi, xj) - 1, 0)
    hi = np.minimum(np.minimum(xi, xj) + 1, g - 1)
    return np.maximum(hi - lo + 1, 0)


def pin_stencil_closed_forms(lib=None, gs=(4, 5, 7)):
    """27-point stencil squared: sizes and (at zero noise) every value have
    closed forms; the per-row entry count is a product of 1-D window counts."""
    for g in gs:
        A = synth.stencil27(g, noise=0.0)
        assert A.nnz == (3 * g - 2) ** 3
        res = oracle.spgemm(A, A, lib=lib)
        assert res.total_products == (9 * g - 10) ** 3
        assert res.nnz == (5 * g - 6) ** 3
        i = np.arange(g ** 3)
        x, y, z = i // (g * g), (i // g) % g, i % g
        per_row = _stencil_c2(x, g) * _stencil_c2(y, g) * _stencil_c2(z, g)
        assert np.array_equal(np.diff(res.row_ptr), per_row)
        rows = np.repeat(i, per_row)
        j = res.col.astype(np.int64)
        xj, yj, zj = j // (g * g), (j // g) % g, j % g
        xi, yi, zi = x[rows], y[rows], z[rows]
        ov = _overlap(xi, xj, g) * _overlap(yi, yj, g) * _overlap(zi, zj, g)
        cheb = np.maximum(np.maximum(np.abs(xi - xj), np.abs(yi - yj)), np.abs(zi - zj))
        deg = (np.minimum(x, 1) + np.minimum(g - 1 - x, 1) + 1) * \
              (np.minimum(y, 1) + np.minimum(g - 1 - y, 1) + 1) * \
              (np.minimum(z, 1) + np.minimum(g - 1 - z, 1) + 1) - 1
        expect = np.where(cheb == 0, 676.0 + deg[rows],
                          np.where(cheb == 1, -52.0 + ov - 2.0, ov.astype(np.float64)))
        assert np.array_equal(res.val, expect)


def pin_identity(lib=None):
    """A*I = A and I*A = A, bit for bit, for canonical A."""
    A = synth.uniform_rows(50, 60, 7, seed=11)
    I60 = synth.from_dense(np.eye(60))
    I50 = synth.from_dense(np.eye(50))
    for left, right in ((A, I60), (I50, A)):
        res = oracle.spgemm(left, right, lib=lib)
        assert np.array_equal(res.row_ptr, A.row_ptr.astype(np.int64))
        assert np.array_equal(res.col, A.col)
        assert np.array_equal(res.val, A.val)


def pin_transpose_symmetry(lib=None):
    """(A B)^T = B^T A^T and A A^T symmetric, bit for bit: with ascending
    columns both sides sum the same products in the same k order."""
    A = synth.erdos_renyi(120, 90, 0.08, seed=21)
    B = synth.erdos_renyi(90, 110, 0.08, seed=22)
    C = oracle.spgemm(A, B, lib=lib)
    D = oracle.spgemm(synth.transpose(B), synth.transpose(A), lib=lib)
    Ct = synth.transpose(synth.CSR(A.rows, B.cols, C.row_ptr, C.col, C.val))
    assert np.array_equal(Ct.row_ptr.astype(np.int64), D.row_ptr)
    assert np.array_equal(Ct.col, D.col)
    assert np.array_equal(Ct.val, D.val)
    S = oracle.spgemm(A, synth.transpose(A), lib=lib)
    St = synth.transpose(synth.CSR(A.rows, A.rows, S.row_ptr, S.col, S.val))
    assert np.array_equal(St.col, S.col) and np.array_equal(St.val, S.val)


def pin_scaling_permutation(lib=None):
    """(2^s A) B = 2^s (A B) and (P A) B = P (A B), bit for bit."""
    A = synth.erdos_renyi(80, 70, 0.1, seed=31)
    B = synth.erdos_renyi(70, 75, 0.1, seed=32)
    C = oracle.spgemm(A, B, lib=lib)
    C8 = oracle.spgemm(A.with_values(A.val * 8.0), B, lib=lib)
    assert np.array_equal(C8.val, C.val * 8.0)
    perm = np.random.default_rng(33).permutation(A.rows)
    rp = A.row_ptr.astype(np.int64)
    lens = np.diff(rp)[perm]
    idx = np.concatenate([np.arange(rp[i], rp[i + 1]) for i in perm])
    prp = np.zeros(A.rows + 1, dtype=np.int64)
    np.cumsum(lens, out=prp[1:])
    PA = synth.CSR(A.rows, A.cols, prp, A.col[idx], A.val[idx])
    PC = oracle.spgemm(PA, B, lib=lib)
    sub = oracle.spgemm(A, B, rows=perm, lib=lib)
    assert np.array_equal(PC.row_ptr, sub.row_ptr)
    assert np.array_equal(PC.col, sub.col) and np.array_equal(PC.val, sub.val)
    # per-row bound: nnz(C_i) <= min(products_i, n)
    assert np.all(np.diff(C.row_ptr) <= np.minimum(C.products, B.cols))


def pin_cancellation_kept(lib=None):
    """An entry whose products cancel exactly stays in the pattern with value 0."""
    A = synth.from_dense(np.array([[1.0, 1.0], [0.0, 2.0]]))
    B = synth.from_dense(np.array([[3.0, 1.0], [-3.0, 0.0]]))
    res = oracle.spgemm(A, B, lib=lib)
    assert list(res.row_ptr) == [0, 2, 3]
    assert list(res.col) == [0, 1, 0]
    assert list(res.val) == [0.0, 1.0, -6.0]


def pin_scipy(lib=None):
    """scipy.sparse's product (a library run as comparator) on workload-shaped
    inputs: same pattern, values within gamma_n * S_ij."""
    import scipy.sparse as sp

    def tosp(M):
        return sp.csr_matrix((M.val.astype(np.float64), M.col, M.row_ptr.astype(np.int64)),
                             shape=(M.rows, M.cols))

    U = synth.uniform_rows()
    S = synth.stencil27(10)
    R = synth.rmat(10)
    for A, B in ((U, U), (S, S), (R, synth.transpose(R))):
        res = oracle.spgemm(A, B, lib=lib)
        C = (tosp(A) @ tosp(B)).tocsr()
        C.sort_indices()
        assert np.array_equal(res.row_ptr, C.indptr.astype(np.int64))
        assert np.array_equal(res.col, C.indices)
        maxterms = int(res.products.max()) if res.products.size else 1
        assert np.all(np.abs(res.val - C.data) <= 2 * gamma(maxterms) * res.sabs)


ALL_PINS = [
    pin_tiny_brute_force,
    pin_dense_matmul,
    pin_integer_exact,
    pin_stencil_closed_forms,
    pin_identity,
    pin_transpose_symmetry,
    pin_scaling_permutation,
    pin_cancellation_kept,
    pin_scipy,
]
