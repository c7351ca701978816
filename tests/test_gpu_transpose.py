"""GPU tests of the device transpose (reap_csr_transpose): bit for bit equal to
the host CSR transpose of the input generators, and products A * A^T built
from it match the oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from parity import compare_full

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def reap():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2004_13907_amd as r
    return r


CASES = {
    "uniform": lambda: synth.uniform_rows(300, 700, 9, seed=1),
    "rmat11": lambda: synth.rmat(11, seed=5),
    "wide_3_passes": lambda: synth.random_tiny(5000, 70000, 0.0008, seed=5, empty_rows=0.2),
    "single_column": lambda: synth.CSR(3, 1, np.array([0, 1, 2, 3], np.int32), np.zeros(3, np.int32),
                                       np.arange(3.0)),
    "empty": lambda: synth.CSR(4, 6, np.zeros(5, np.int32), np.zeros(0, np.int32), np.zeros(0)),
    "stencil9": lambda: synth.stencil27(9),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("dtype,index", [("f64", "i32"), ("f32", "i32"), ("f64", "i64")])
def test_transpose_bit_exact(reap, name, dtype, index):
    A = CASES[name]()
    npdt = np.float64 if dtype == "f64" else np.float32
    tdt = torch.float64 if dtype == "f64" else torch.float32
    tidx = torch.int64 if index == "i64" else torch.int32
    A = A.astype(npdt)
    say("transpose", name, dtype, index, A.rows, A.cols, A.nnz)
    dA = reap.DeviceCSR.from_host(A, dtype=tdt, index_dtype=tidx)
    T = reap.transpose(dA)
    torch.cuda.synchronize()
    rp, col, val = T.to_host()
    ref = synth.transpose(A)
    assert T.rows == A.cols and T.cols == A.rows
    assert np.array_equal(rp.astype(np.int64), ref.row_ptr.astype(np.int64))
    assert np.array_equal(col, ref.col)
    assert np.array_equal(val, ref.val.astype(npdt))


def test_product_with_device_transpose(reap):
    """A * A^T with A^T from the device transpose, against the oracle."""
    A = synth.rmat(11, seed=9).astype(np.float32)
    say("rmat11 A*A^T with the device transpose")
    dA = reap.DeviceCSR.from_host(A, dtype=torch.float32)
    dT = reap.transpose(dA)
    C = reap.spgemm(dA, dT)
    torch.cuda.synchronize()
    rp, col, val = C.to_host()
    compare_full(oracle.spgemm(A, synth.transpose(A)), rp, col, val, np.float32, "A*A^T device transpose")


def test_transpose_full_size_rmat(reap):
    A = synth.rmat(18)
    say("rmat18 transpose")
    dA = reap.DeviceCSR.from_host(A, dtype=torch.float32)
    T = reap.transpose(dA)
    torch.cuda.synchronize()
    rp, col, val = T.to_host()
    ref = synth.transpose(A)
    assert np.array_equal(rp.astype(np.int64), ref.row_ptr.astype(np.int64))
    assert np.array_equal(col, ref.col)
    assert np.array_equal(val, ref.val.astype(np.float32))
