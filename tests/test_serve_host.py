"""Host-only tests of the serving loop's admission and error handling.

The device work is replaced by a stand-in batch (symbolic returns the sizes
the request carries, numeric sleeps or raises), so these run without a GPU:
the accounted peak never exceeds the HBM budget, a request larger than the
whole budget is rejected while the loop goes on, and an error raised inside
an admitted batch reaches run() instead of leaving a slot that waits for
memory blocked forever."""
from __future__ import annotations

import contextlib
import threading
import time
from types import SimpleNamespace

import pytest

torch = pytest.importorskip("torch")

from paper_2004_13907_amd.serve import Request, Server  # noqa: E402


class FakeBatch:
    """Stand-in for paper_2004_13907_amd.Batch: sizes come from the operands."""

    ws_per_row = 16

    def __init__(self, dtype, c_index_dtype, stream=None, **options):
        self.dtype = dtype
        self.workspace_bytes = 0
        self.products = []
        self.nnz = []

    def workspace_query(self, As, Bs):
        return max(self.workspace_bytes, self.ws_per_row * sum(A.rows for A in As))

    def symbolic(self, As, Bs, fresh=False):
        time.sleep(0.001)
        self.workspace_bytes = self.workspace_query(As, Bs)
        self.nnz = [A.nnz_c for A in As]
        self.products = [2 * A.nnz_c for A in As]
        return list(self.nnz)

    def numeric(self, As, Bs):
        for A in As:
            if A.fail:
                raise RuntimeError("numeric failed (planted)")
        time.sleep(0.002 * len(As))
        return [None for _ in As]

    def close(self):
        pass


class FakeStream:
    def synchronize(self):
        pass


class HostServer(Server):
    batch_class = FakeBatch

    def _new_stream(self):
        return FakeStream()

    def _on_stream(self, stream):
        return contextlib.nullcontext()

    def _device_sync(self):
        pass


def _op(rows, nnz_c, fail=False):
    return SimpleNamespace(rows=rows, nnz_c=nnz_c, fail=fail, dtype=torch.float64)


def _footprint(rows, nnz_c):
    # int64 row pointers + int32 columns + FP64 values + the stand-in's workspace
    return (rows + 1) * 8 + nnz_c * 12 + FakeBatch.ws_per_row * rows


def _run_with_deadline(srv, reqs, seconds=20.0):
    out = {}

    def body():
        try:
            out["stats"] = srv.run(reqs)
        except BaseException as e:  # noqa: BLE001
            out["error"] = e

    t = threading.Thread(target=body, daemon=True)
    t.start()
    t.join(seconds)
    assert not t.is_alive(), "the serving loop did not finish (deadlock)"
    return out


def test_budget_is_never_exceeded():
    sizes = [(100 + 37 * i, 2_000 + 1_500 * (i % 7)) for i in range(60)]
    budget = 3 * max(_footprint(r, z) for r, z in sizes)
    reqs = [Request(i, _op(r, z), _op(r, z), arrival=0.0005 * i) for i, (r, z) in enumerate(sizes)]
    srv = HostServer(slots=3, hbm_budget_bytes=budget, max_batch=6)
    out = _run_with_deadline(srv, reqs)
    st = out["stats"]
    assert st.requests == len(reqs) and st.rejected == 0
    assert all(r.status == "ok" for r in reqs)
    assert st.peak_bytes <= budget
    assert st.resymbolic + st.waits_for_memory > 0, "the budget never constrained admission"


def test_request_larger_than_the_budget_is_rejected():
    small = [(64, 1_000)] * 8
    reqs = [Request(i, _op(r, z), _op(r, z), arrival=0.0) for i, (r, z) in enumerate(small)]
    big = Request(99, _op(64, 10_000_000), _op(64, 10_000_000), arrival=0.0)
    reqs.insert(3, big)
    budget = 20 * _footprint(64, 1_000)
    srv = HostServer(slots=2, hbm_budget_bytes=budget, max_batch=4)
    st = _run_with_deadline(srv, reqs)["stats"]
    assert big.status == "rejected" and "budget" in big.error
    assert st.rejected == 1 and st.requests == len(reqs) - 1
    assert all(r.status == "ok" for r in reqs if r is not big)
    assert st.peak_bytes <= budget


def test_error_in_an_admitted_batch_does_not_block_a_waiting_slot():
    # request 0 fills most of the budget and fails inside numeric; request 1
    # arrives while it runs and has to wait for its memory
    budget = int(1.5 * _footprint(64, 100_000))
    reqs = [Request(0, _op(64, 100_000, fail=True), _op(64, 100_000), arrival=0.0),
            Request(1, _op(64, 100_000), _op(64, 100_000), arrival=0.0005)]
    srv = HostServer(slots=2, hbm_budget_bytes=budget, max_batch=1)
    out = _run_with_deadline(srv, reqs)
    assert "error" in out and "planted" in str(out["error"])


def test_served_requests_are_stamped():
    reqs = [Request(i, _op(10, 50), _op(10, 50), arrival=0.0) for i in range(5)]
    st = _run_with_deadline(HostServer(slots=1, hbm_budget_bytes=1e9, max_batch=8), reqs)["stats"]
    assert st.requests == 5 and st.batches >= 1
    for r in reqs:
        assert r.status == "ok" and r.done >= r.admitted >= r.arrival and r.nnz == 50
