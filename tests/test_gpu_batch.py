"""GPU parity of the batched entry points (reap_spgemm_batch_symbolic /
reap_spgemm_batch_numeric): many independent products in one launch per
kernel, eagerly and captured in HIP graphs, each product against the oracle."""
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


def _mixed_products(npdt):
    """Products of every kind in one batch: banded, uniform, an empty A, long
    rows, a skewed A*A^T and an irregular pair with duplicates and unsorted
    columns."""
    out = []
    S = synth.stencil27(6)
    out.append((S, S))
    U = synth.uniform_rows(300, 300, 8, seed=5)
    out.append((U, U))
    out.append((synth.CSR(0, 40, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0)),
                synth.uniform_rows(40, 25, 3, seed=6)))
    E = synth.erdos_renyi(700, 700, 0.06, seed=7)
    out.append((E, E))
    R = synth.rmat(9, seed=8)
    out.append((R, synth.transpose(R)))
    A = synth.random_tiny(400, 300, 0.03, seed=9, allow_duplicates=True, unsorted=True, empty_rows=0.1)
    B = synth.random_tiny(300, 500, 0.04, seed=10, empty_rows=0.1)
    out.append((A, B))
    return [(a.astype(npdt), b.astype(npdt)) for a, b in out]


def _device(reap, pairs, tdt):
    dA = [reap.DeviceCSR.from_host(a, dtype=tdt) for a, _ in pairs]
    dB = [reap.DeviceCSR.from_host(b, dtype=tdt) for _, b in pairs]
    return dA, dB


def _check_all(pairs, results, npdt, label):
    for q, ((A, B), C) in enumerate(zip(pairs, results)):
        rp, col, val = C.to_host()
        ref = oracle.spgemm(A, B)
        compare_full(ref, rp, col, val, npdt, "%s product %d" % (label, q))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_mixed_eager(reap, dtype):
    tdt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    pairs = _mixed_products(npdt)
    say("batch mixed eager", dtype, len(pairs), "products")
    dA, dB = _device(reap, pairs, tdt)
    with reap.Batch(tdt) as b:
        nnz = b.symbolic(dA, dB)
        res = b.numeric(dA, dB)
        b.synchronize()
        assert nnz == [oracle.spgemm(A, B, with_values=False).nnz for A, B in pairs]
        _check_all(pairs, res, npdt, "eager " + dtype)


def test_batch_forced_long_rows(reap):
    """Every row of every product through the long-row kernels, with small
    column segments."""
    pairs = _mixed_products(np.float64)
    say("batch all rows long")
    dA, dB = _device(reap, pairs, torch.float64)
    with reap.Batch(torch.float64, wave_max_products=-1, group_lds_span=96) as b:
        b.symbolic(dA, dB)
        res = b.numeric(dA, dB)
        b.synchronize()
        _check_all(pairs, res, np.float64, "all long")


@pytest.mark.parametrize("slots", [512, 1024])
def test_batch_hash_rows(reap, slots):
    """Every row the bitmap would take goes to the wavefront hash class instead
    (512- and 1024-slot tables, argument tables of a batch), plus a product
    whose rows of 400 products need the larger table."""
    pairs = _mixed_products(np.float64)
    pairs.append((synth.uniform_rows(200, 20000, 20, seed=13), synth.uniform_rows(20000, 40000, 20, seed=14)))
    say("batch hash rows", slots)
    dA, dB = _device(reap, pairs, torch.float64)
    with reap.Batch(torch.float64, wave_max_span=-1, wave_hash_slots=slots) as b:
        b.symbolic(dA, dB)
        res = b.numeric(dA, dB)
        b.synchronize()
        st = b.plan.bin_stats()
        assert st["wave_bitmap"] == 0 and st["wave_hash"] > 0, st
        _check_all(pairs, res, np.float64, "hash %d" % slots)


def test_batch_of_one_matches_single(reap):
    E = synth.erdos_renyi(900, 900, 0.03, seed=11)
    say("batch of one vs single call")
    dE = reap.DeviceCSR.from_host(E)
    single = reap.spgemm(dE, dE)
    with reap.Batch(torch.float64) as b:
        b.symbolic([dE], [dE])
        (C,) = b.numeric([dE], [dE])
        b.synchronize()
    r1, c1, _ = single.to_host()
    r2, c2, v2 = C.to_host()
    assert np.array_equal(r1, r2) and np.array_equal(c1, c2)
    compare_full(oracle.spgemm(E, E), r2, c2, v2, np.float64, "batch of one")


def test_batch_graph_replays(reap):
    """Captured passes replayed several times, with eager work of the program
    between the replays; every replay is checked against the oracle, and then
    new values on the same patterns are multiplied by the captured numeric
    graph."""
    pairs = _mixed_products(np.float64)
    dA, dB = _device(reap, pairs, torch.float64)
    refs = [oracle.spgemm(A, B) for A, B in pairs]
    with reap.Batch(torch.float64, graph=True) as b:
        for rep in range(3):
            say("batch graph replay", rep)
            b.symbolic(dA, dB)
            res = b.numeric(dA, dB)
            b.synchronize()
            junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)  # eager work between replays
            float((junk * 2).sum())
            for q, (C, ref) in enumerate(zip(res, refs)):
                rp, col, val = C.to_host()
                compare_full(ref, rp, col, val, np.float64, "graph rep %d product %d" % (rep, q))
        rng = np.random.default_rng(12)
        new_pairs, nA = [], []
        for (A, B), da in zip(pairs, dA):
            vals = rng.uniform(-1, 1, size=A.nnz)
            new_pairs.append((synth.CSR(A.rows, A.cols, A.row_ptr, A.col, vals), B))
            nA.append(reap.DeviceCSR(da.rows, da.cols, da.row_ptr, da.col,
                                     torch.from_numpy(vals).to("cuda")))
        say("batch graph numeric with new values")
        res = b.numeric(nA, dB)
        b.synchronize()
        _check_all(new_pairs, res, np.float64, "graph new values")
