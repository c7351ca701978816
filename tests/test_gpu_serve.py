"""GPU tests of the serving loop: every request served in a mix of concurrent,
continuously batched requests gives the result it gives alone (pattern bit
for bit, values within the per-entry tolerance of the oracle), also when the
HBM budget forces batches to shrink and requests to wait for memory."""
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


def _pool(reap, served_sizes=False):
    """(kind, host A, host B, device A, device B) for a small mix of jobs; with
    ``served_sizes`` the mix also holds jobs at the served workload's sizes
    (stencil g = 16, R-MAT scales 13 and 14, uniform-random m = 4096)."""
    jobs = []
    for g in (6, 9, 12) + ((16,) if served_sizes else ()):
        S = synth.stencil27(g, seed=g)
        jobs.append(("stencil", S, S, torch.float64))
    for sc in (8, 9, 10) + ((13, 14) if served_sizes else ()):
        R = synth.rmat(sc, seed=sc).astype(np.float32)
        jobs.append(("rmat", R, synth.transpose(R), torch.float32))
    for m, d in ((500, 0.03), (1500, 0.01)) + (((4096, 0.005),) if served_sizes else ()):
        A = synth.erdos_renyi(m, m, d, seed=m)
        B = synth.erdos_renyi(m, m, d, seed=m + 1)
        jobs.append(("uniform", A, B, torch.float64))
    out = []
    for kind, A, B, tdt in jobs:
        dA = reap.DeviceCSR.from_host(A, dtype=tdt)
        dB = reap.DeviceCSR.from_host(B, dtype=tdt)
        out.append((kind, A, B, dA, dB))
    return out


def _requests(reap, pool, n, qps, seed):
    from paper_2004_13907_amd.serve import Request
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / qps, size=n))
    picks = rng.integers(0, len(pool), size=n)
    return [Request(i, pool[p][3], pool[p][4], float(t[i]), kind=pool[p][0]) for i, p in enumerate(picks)], picks


def _check_against_alone(reap, pool, reqs, picks):
    alone = {}
    refs = {}
    for i, p in enumerate(picks):
        kind, A, B, dA, dB = pool[p]
        assert reqs[i].status == "ok", "request %d: %s %s" % (i, reqs[i].status, reqs[i].error)
        if p not in alone:
            C = reap.spgemm(dA, dB, c_index_dtype=torch.int64)
            torch.cuda.synchronize()
            alone[p] = C.to_host()
            refs[p] = oracle.spgemm(A, B)
        r = reqs[i]
        rp, col, val = r.C.to_host()
        arp, acol, aval = alone[p]
        assert np.array_equal(rp, arp) and np.array_equal(col, acol), "request %d: pattern differs from alone" % i
        ref = refs[p]
        tol = tolerance(val.dtype)
        scale = np.maximum(ref.sabs, np.finfo(np.float64).tiny)
        diff = np.abs(val.astype(np.float64) - aval.astype(np.float64)) / scale
        assert diff.max(initial=0.0) <= 2 * tol, "request %d: mix vs alone %.3e" % (i, diff.max())
        compare_full(ref, rp, col, val, val.dtype, "request %d (%s)" % (i, kind))


def _footprints(reap, pool):
    """Device bytes of each job served alone: C (columns + values), int64 row
    pointers and the workspace a fresh plan holds after its symbolic pass
    (the serving loop reserves the library's upper bound before that pass and
    keeps only what was really allocated)."""
    foot = []
    for kind, A, B, dA, dB in pool:
        ref = oracle.spgemm(A, B, with_values=False)
        with reap.Batch(dA.dtype, torch.int64) as b:
            assert b.workspace_query([dA], [dB]) >= 0
            b.symbolic([dA], [dB])
            ws = b.workspace_bytes
        foot.append(ref.nnz * (4 + dA.val.element_size()) + (A.rows + 1) * 8 + ws)
    return foot


def test_served_mix_matches_alone(reap):
    """A mix that includes jobs at the served workload's sizes: every request
    gives the same result in the mix as alone, and the oracle's."""
    from paper_2004_13907_amd.serve import Server
    pool = _pool(reap, served_sizes=True)
    reqs, picks = _requests(reap, pool, 40, qps=4000.0, seed=21)
    say("served mix: 40 requests, 3 slots, jobs up to R-MAT 14 / stencil 16 / uniform 4096")
    srv = Server(slots=3, hbm_budget_bytes=8e9, max_batch=6)
    try:
        st = srv.run(reqs)
    finally:
        srv.close()
    assert st.requests == 40 and all(r.done is not None and r.done >= r.arrival for r in reqs)
    assert st.batches < 40, "requests that arrive together are batched"
    assert st.peak_bytes <= st.budget_bytes
    _check_against_alone(reap, pool, reqs, picks)


def test_served_memory_admission(reap):
    """A budget about twice the largest single request's footprint: batches
    must shrink or wait for memory, the accounted peak stays within the
    budget, and every result still matches."""
    from paper_2004_13907_amd.serve import Server
    pool = _pool(reap, served_sizes=True)
    foot = _footprints(reap, pool)
    reqs, picks = _requests(reap, pool, 30, qps=1e5, seed=22)
    budget = 2.2 * max(foot)
    say("served under a tight HBM budget (%.1f MB)" % (budget / 1e6))
    srv = Server(slots=3, hbm_budget_bytes=budget, max_batch=8)
    try:
        st = srv.run(reqs)
    finally:
        srv.close()
    assert st.rejected == 0 and st.requests == 30
    assert st.resymbolic + st.waits_for_memory > 0, "the budget never constrained admission"
    assert st.peak_bytes <= budget, "accounted peak %d above the budget %d" % (st.peak_bytes, budget)
    _check_against_alone(reap, pool, reqs, picks)


def test_served_rejects_what_cannot_fit(reap):
    """A request whose footprint alone exceeds the budget is rejected with a
    status; the requests around it are served and match."""
    from paper_2004_13907_amd.serve import Server
    pool = _pool(reap)
    foot = _footprints(reap, pool)
    big = int(np.argmax(foot))
    budget = 0.9 * foot[big]
    small = [i for i, f in enumerate(foot) if f * 2 < budget]
    assert small, "no job small enough for the budget"
    from paper_2004_13907_amd.serve import Request
    picks = [small[i % len(small)] for i in range(6)]
    reqs = [Request(i, pool[p][3], pool[p][4], 0.0, kind=pool[p][0]) for i, p in enumerate(picks)]
    reqs.append(Request(6, pool[big][3], pool[big][4], 0.0, kind=pool[big][0]))
    say("served with one request above the budget (%.1f MB)" % (budget / 1e6))
    srv = Server(slots=2, hbm_budget_bytes=budget, max_batch=4)
    try:
        st = srv.run(reqs)
    finally:
        srv.close()
    assert reqs[6].status == "rejected" and st.rejected == 1
    assert st.peak_bytes <= budget
    _check_against_alone(reap, pool, reqs[:6], picks)
