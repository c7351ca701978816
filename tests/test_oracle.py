"""The oracle checked against its independent pins (CPU only)."""
import numpy as np
import pytest

import oracle
import synth
from pins import ALL_PINS


@pytest.mark.parametrize("pin", ALL_PINS, ids=[p.__name__ for p in ALL_PINS])
def test_pin(pin, oracle_lib):
    pin()


def test_threads_bit_identical(oracle_lib):
    A = synth.rmat(11)
    B = synth.transpose(A)
    one = oracle.spgemm(A, B, threads=1)
    many = oracle.spgemm(A, B, threads=4)
    assert np.array_equal(one.row_ptr, many.row_ptr)
    assert np.array_equal(one.col, many.col)
    assert np.array_equal(one.val, many.val)
    assert np.array_equal(one.sabs, many.sabs)


def test_row_subset_matches_full(oracle_lib):
    A = synth.uniform_rows(300, 200, 6, seed=5)
    B = synth.uniform_rows(200, 250, 4, seed=6)
    full = oracle.spgemm(A, B)
    rows = np.array([7, 0, 299, 7, 150])
    sub = oracle.spgemm(A, B, rows=rows)
    for r, i in enumerate(rows):
        a, b = full.row_ptr[i], full.row_ptr[i + 1]
        c, d = sub.row_ptr[r], sub.row_ptr[r + 1]
        assert np.array_equal(full.col[a:b], sub.col[c:d])
        assert np.array_equal(full.val[a:b], sub.val[c:d])


def test_empty_and_degenerate(oracle_lib):
    E = synth.CSR(0, 5, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    B = synth.uniform_rows(5, 4, 2, seed=1)
    r = oracle.spgemm(E, B)
    assert r.nnz == 0 and r.row_ptr.tolist() == [0]
    Z = synth.CSR(3, 5, np.zeros(4, np.int32), np.zeros(0, np.int32), np.zeros(0))
    r = oracle.spgemm(Z, B)
    assert r.nnz == 0 and r.row_ptr.tolist() == [0, 0, 0, 0]
    with pytest.raises(ValueError):
        oracle.spgemm(B, B)


def test_uniform_config_products(oracle_lib):
    A = synth.uniform_rows()
    r = oracle.spgemm(A, A, with_values=False)
    assert r.total_products == 200_000
    assert np.all(r.products == 100)


def test_fp32_promotion_exact(oracle_lib):
    """FP32 inputs: each product of two binary32 values is exact in binary64,
    so single-term entries equal the exact product."""
    A = synth.uniform_rows(64, 64, 1, seed=9, dtype=np.float32)
    B = synth.uniform_rows(64, 64, 1, seed=10, dtype=np.float32)
    r = oracle.spgemm(A, B)
    for i in range(64):
        k = A.col[i]
        assert r.val[i] == float(A.val[i]) * float(B.val[k])
        assert r.col[i] == B.col[k]
