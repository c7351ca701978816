"""Generator shapes (CPU only)."""
import numpy as np

import synth


def _canonical(A):
    rp = A.row_ptr.astype(np.int64)
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == A.col.size == A.val.size
    for i in range(0, A.rows, max(1, A.rows // 97)):
        c = A.col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0)
    assert A.col.size == 0 or (A.col.min() >= 0 and A.col.max() < A.cols)


def test_uniform_rows_shape():
    A = synth.uniform_rows()
    _canonical(A)
    assert A.rows == A.cols == 2000 and A.nnz == 20000
    assert np.all(A.row_lengths() == 10)
    assert A.val.min() >= -1 and A.val.max() <= 1 and A.val.dtype == np.float64
    B = synth.uniform_rows()
    assert np.array_equal(A.col, B.col) and np.array_equal(A.val, B.val)


def test_stencil_shape():
    for g in (3, 4, 9):
        A = synth.stencil27(g)
        _canonical(A)
        assert A.rows == g ** 3 and A.nnz == (3 * g - 2) ** 3
    A = synth.stencil27(6, noise=0.0)
    i = np.repeat(np.arange(A.rows), A.row_lengths())
    assert np.all(A.val[A.col == i] == 26.0) and np.all(A.val[A.col != i] == -1.0)
    A = synth.stencil27(6)
    dev = np.abs(A.val - np.where(A.col == i, 26.0, -1.0))
    assert dev.max() <= 0.01 and dev.max() > 0


def test_rmat_shape():
    A = synth.rmat(12)
    _canonical(A)
    assert A.rows == A.cols == 4096
    assert A.nnz <= 16 * 4096 and A.nnz > 0.8 * 16 * 4096
    assert A.val.dtype == np.float32 and A.val.min() > 0 and A.val.max() <= 1
    lens = A.row_lengths()
    assert lens[0] == lens.max()          # vertex 0 is the heaviest hub (a > b, c, d)
    T = synth.transpose(A)
    _canonical(T)
    assert T.nnz == A.nnz


def test_erdos_renyi_shape():
    A = synth.erdos_renyi(3000, 2500, 4e-3, seed=3)
    _canonical(A)
    assert abs(A.nnz - 3000 * 2500 * 4e-3) < 6 * np.sqrt(3000 * 2500 * 4e-3)


def test_batched_and_served_specs():
    specs = synth.batched_set()
    assert len(specs) == 512
    ms = np.array([s.m for s in specs])
    assert ms.min() >= 1024 and ms.max() <= 65536 and 5000 < np.median(ms) < 13000
    ds = np.array([s.density for s in specs])
    assert ds.min() >= 1e-3 and ds.max() <= 1e-2
    jobs = synth.served_jobs(400, qps=10.0)
    kinds = [j.kind for j in jobs]
    assert 0.3 < kinds.count("stencil") / 400 < 0.5 and 0.1 < kinds.count("uniform") / 400 < 0.3
    t = np.array([j.arrival_s for j in jobs])
    assert np.all(np.diff(t) >= 0) and 20 < t[-1] < 60
