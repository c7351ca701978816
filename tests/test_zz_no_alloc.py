"""GPU tests of reap_spgemm_symbolic_noalloc (the allocation-free symbolic
call, workspace in the library's static scratch) through the C ABI: its
results, with the unchanged numeric call, equal those of reap_spgemm_symbolic
+ numeric and the oracle's, on two calls in a row with the second smaller
(the scratch keeps the first call's contents), for FP64 and FP32 products,
long rows included and FP32 long rows that need device-memory accumulators;
an oversize product is refused before any device work; the plan returns to
its own workspace afterwards."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from parity import compare_full, tolerance

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


def _run(reap, plan, dA, dB, noalloc):
    from paper_2004_13907_amd import _capi
    rp = torch.empty(dA.rows + 1, dtype=plan.c_index_dtype, device="cuda")
    if noalloc:
        st, nnz, prods = reap.reap_spgemm_symbolic_noalloc(plan.handle, dA, dB, rp)
    else:
        st, nnz, prods, _ = reap.reap_spgemm_symbolic(plan.handle, dA, dB, rp)
    assert st == _capi.REAP_OK, reap.reap_status_string(st)
    col = torch.empty(nnz, dtype=torch.int32, device="cuda")
    val = torch.empty(nnz, dtype=plan.dtype, device="cuda")
    st = reap.reap_spgemm_numeric(plan.handle, dA, dB, rp, col, val)
    assert st == _capi.REAP_OK, reap.reap_status_string(st)
    torch.cuda.synchronize()
    stats = plan.bin_stats()
    return rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy(), prods, stats


def _pairs(kind):
    """(label, A, B, plan options): the first pair larger than the second."""
    if kind == "f64":
        return [("stencil 20", synth.stencil27(20), None, {}),
                ("stencil 9", synth.stencil27(9), None, {})]
    if kind == "f32":
        R10 = synth.rmat(10).astype(np.float32)
        R8 = synth.rmat(8).astype(np.float32)
        return [("rmat 10 A*A^T", R10, synth.transpose(R10), {}),
                ("rmat 8 A*A^T", R8, synth.transpose(R8), {})]
    # FP32 long rows over B rows out of column order, cut into 256-slot
    # chunks: the FP64 accumulators live in the static scratch too
    A1 = synth.erdos_renyi(300, 2000, 0.05, seed=71, dtype=np.float32)
    B1 = synth.random_tiny(2000, 20000, 0.03, seed=72, dtype=np.float32, unsorted=True)
    A2 = synth.erdos_renyi(120, 2000, 0.05, seed=73, dtype=np.float32)
    return [("unsorted long rows 300", A1, B1, {"group_lds_values": 256}),
            ("unsorted long rows 120", A2, B1, {"group_lds_values": 256})]


@pytest.mark.parametrize("kind", ["f64", "f32", "f32_unsorted_long"])
def test_noalloc_matches_regular_entry_point(reap, kind):
    tdt = torch.float64 if kind == "f64" else torch.float32
    npdt = np.float64 if kind == "f64" else np.float32
    pairs = _pairs(kind)
    opts = pairs[0][3]
    with reap.Plan(tdt, torch.int32, **opts) as plan_na, reap.Plan(tdt, torch.int32, **opts) as plan_reg:
        for label, A, B, _ in pairs:           # two calls in a row, the second smaller
            B = A if B is None else B
            say("noalloc", kind, label)
            dA = reap.DeviceCSR.from_host(A, dtype=tdt)
            dB = dA if B is A else reap.DeviceCSR.from_host(B, dtype=tdt)
            rp, col, val, prods, st_na = _run(reap, plan_na, dA, dB, noalloc=True)
            rrp, rcol, rval, rprods, st_reg = _run(reap, plan_reg, dA, dB, noalloc=False)
            assert np.array_equal(rp, rrp) and np.array_equal(col, rcol), label
            assert prods == rprods
            for key in ("empty", "wave_bitmap", "wave_hash", "group", "long_segments_lds",
                        "long_segments_chunked", "long_segments_device"):
                assert st_na[key] == st_reg[key], (label, key, st_na, st_reg)
            ref = oracle.spgemm(A, B)
            compare_full(ref, rp, col, val, npdt, "noalloc " + label)
            scale = np.maximum(ref.sabs, np.finfo(np.float64).tiny)
            diff = np.abs(val.astype(np.float64) - rval.astype(np.float64)) / scale
            assert diff.max(initial=0.0) <= 2 * tolerance(npdt), label
            if kind == "f32_unsorted_long":
                assert st_na["long_segments_device"] > 0, st_na
        # the plan goes back to its own workspace for a regular call
        label, A, B, _ = pairs[1]
        B = A if B is None else B
        dA = reap.DeviceCSR.from_host(A, dtype=tdt)
        dB = dA if B is A else reap.DeviceCSR.from_host(B, dtype=tdt)
        rp, col, val, _, _ = _run(reap, plan_na, dA, dB, noalloc=False)
        compare_full(oracle.spgemm(A, B), rp, col, val, npdt, "regular call after noalloc " + label)


def test_noalloc_refuses_oversize(reap):
    from paper_2004_13907_amd import _capi
    m = 4_000_000                                   # ~88 MB of per-row workspace > 64 MiB
    say("noalloc oversize: %d rows" % m)
    A = reap.DeviceCSR(m, 10, torch.zeros(m + 1, dtype=torch.int32, device="cuda"),
                       torch.zeros(0, dtype=torch.int32, device="cuda"),
                       torch.zeros(0, dtype=torch.float64, device="cuda"))
    B = reap.DeviceCSR(10, 10, torch.zeros(11, dtype=torch.int32, device="cuda"),
                       torch.zeros(0, dtype=torch.int32, device="cuda"),
                       torch.zeros(0, dtype=torch.float64, device="cuda"))
    with reap.Plan(torch.float64) as plan:
        rp = torch.empty(m + 1, dtype=torch.int32, device="cuda")
        st, _, _ = reap.reap_spgemm_symbolic_noalloc(plan.handle, A, B, rp)
        assert st == _capi.REAP_ERR_TOO_LARGE
        rp2, nnz, _ = plan.symbolic(A, B)             # the regular call allocates and succeeds
        assert nnz == 0


def test_noalloc_allocates_no_device_memory(reap):
    """Free device memory is unchanged across the allocation-free symbolic
    call and the numeric call after it (the stencil 64^3 product: the plan's
    own workspace would take about 5.8 MB), while a regular symbolic call on
    a fresh plan takes its workspace."""
    from paper_2004_13907_amd import _capi
    A = synth.stencil27(64)
    dA = reap.DeviceCSR.from_host(A)
    rp = torch.empty(A.rows + 1, dtype=torch.int32, device="cuda")
    say("noalloc: device memory around the calls (stencil 64)")
    with reap.Plan(torch.float64) as plan:
        st, nnz, _ = reap.reap_spgemm_symbolic_noalloc(plan.handle, dA, dA, rp)   # warm-up launches
        assert st == _capi.REAP_OK
        col = torch.empty(nnz, dtype=torch.int32, device="cuda")
        val = torch.empty(nnz, dtype=torch.float64, device="cuda")
        assert reap.reap_spgemm_numeric(plan.handle, dA, dA, rp, col, val) == _capi.REAP_OK
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        st, nnz2, _ = reap.reap_spgemm_symbolic_noalloc(plan.handle, dA, dA, rp)
        assert st == _capi.REAP_OK and nnz2 == nnz
        assert reap.reap_spgemm_numeric(plan.handle, dA, dA, rp, col, val) == _capi.REAP_OK
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        assert free0 - free1 < (1 << 20), "device memory fell by %d bytes" % (free0 - free1)
        assert nnz == 30_959_144
    with reap.Plan(torch.float64) as plan:
        free2 = torch.cuda.mem_get_info()[0]
        st, _, _, ws = reap.reap_spgemm_symbolic(plan.handle, dA, dA, rp)
        torch.cuda.synchronize()
        free3 = torch.cuda.mem_get_info()[0]
        assert st == _capi.REAP_OK and ws > 5_000_000 and free2 - free3 >= ws
