"""Serving loop for SpGEMM requests with continuous batching.

Requests (operands already in device memory) arrive over time.  The
scheduler thread moves arrived requests to a queue and, whenever a slot is
idle, hands it a batch: the oldest waiting request and the following ones
with the same value type, up to `max_batch`.  Each slot owns a stream, one
plan per value type and a host worker thread, which
  1. reserves the symbolic pass's own device memory -- the batch's C row
     pointers and whatever the plan's workspace must grow by (asked of the
     library before anything is allocated) -- against the HBM budget,
  2. runs the batched symbolic pass (blocking only its own thread: the C
     calls release the interpreter lock, and the wait is on its own stream),
  3. reserves C's columns and values, now known exactly,
  4. enqueues the numeric pass, waits for its own stream, stamps every
     request of the batch with its completion time and releases the row
     pointers and C (the results belong to the caller from then on).
When a reservation does not fit, a batch of several requests gives its newest
half back to the queue and retries with the rest; a single request waits for
memory while other batches are in flight, and is rejected (status
"rejected", the loop goes on) when it cannot fit even with nothing else in
flight.  The plans' workspaces stay allocated between batches and are
counted as used for as long as they exist, so the accounted peak -- resident
workspaces plus every in-flight batch's row pointers and C -- never exceeds
the budget.  Batches on different slots overlap on the device and on the
host.  Latency is arrival to the completion of the request's batch on the
device, as seen by the host.

The paper overlaps the CPU's preparation of the next work with the
accelerator's computation (Section II); here the symbolic pass and host work
of one batch overlap the numeric pass of another."""
from __future__ import annotations

import queue as _queue
import threading
import time
from dataclasses import dataclass, field

import torch

from . import Batch, DeviceCSR


@dataclass
class Request:
    rid: int
    A: DeviceCSR
    B: DeviceCSR
    arrival: float                    # seconds after the start of the trace
    kind: str = ""
    # filled in by the server
    status: str = "pending"           # "ok" or "rejected"
    error: str = ""
    admitted: float | None = None
    done: float | None = None
    C: DeviceCSR | None = None
    products: int = 0
    nnz: int = 0
    batch_size: int = 0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class ServeStats:
    requests: int                     # served (status "ok")
    seconds: float                    # first arrival to last completion
    products: int
    gflops: float
    p50_ms: float
    p99_ms: float
    mean_batch: float
    batches: int
    peak_bytes: int                   # accounted device bytes: resident workspaces + in-flight batches
    budget_bytes: int
    resymbolic: int                   # batches shrunk to fit the budget
    waits_for_memory: int
    rejected: int = 0
    per_kind: dict = field(default_factory=dict)


def _pct(sorted_vals, q):
    return sorted_vals[min(len(sorted_vals) - 1, int(q * len(sorted_vals)))]


class Server:
    # Two slots overlap one batch's host work and symbolic pass with another's
    # numeric pass.  Measured on an MI355X with the served job mix at 0.8x of
    # the closed-loop rate: one or two slots keep up (two: p50 82 ms, p99
    # 0.4 s), four fall behind (p50 2 s).
    batch_class = Batch                       # replaced by a stand-in in the host-only tests

    def __init__(self, slots: int = 2, hbm_budget_bytes: float = 64e9, max_batch: int = 16,
                 keep_results: bool = True, c_index_dtype=torch.int64, **options):
        self.nslots = slots
        self.budget = int(hbm_budget_bytes)
        self.max_batch = max_batch
        self.keep_results = keep_results
        self.c_index_dtype = c_index_dtype
        self.options = options
        self.streams = [self._new_stream() for _ in range(slots)]
        self.batches = [dict() for _ in range(slots)]   # value dtype -> Batch on that slot's stream
        self.idx_bytes = torch.tensor([], dtype=c_index_dtype).element_size()
        self.resident = {}                              # (slot, dtype) -> workspace bytes the plan holds
        # an idle slot keeps at most this much plan workspace between batches,
        # so that resident workspaces take at most a quarter of the budget
        self.keep_cap = self.budget // (4 * max(1, slots))
        self._st = None

    # -- device hooks (host-only tests replace these) ------------------------------
    def _new_stream(self):
        return torch.cuda.Stream()

    def _on_stream(self, stream):
        return torch.cuda.stream(stream)

    def _device_sync(self):
        torch.cuda.synchronize()

    def close(self):
        for d in self.batches:
            for b in d.values():
                b.close()
        self.batches = [dict() for _ in range(self.nslots)]
        self.resident = {}

    # -- worker side -------------------------------------------------------------
    def _batch(self, slot, dtype):
        b = self.batches[slot].get(dtype)
        if b is None:
            b = self.batch_class(dtype, self.c_index_dtype, stream=self.streams[slot], **self.options)
            self.batches[slot][dtype] = b
        return b

    def _reject(self, r, why, st):
        r.status = "rejected"
        r.error = why
        r.done = time.perf_counter() - st["t0"]
        with st["cv"]:
            st["rejected"].append(r)

    def _run_batch(self, slot, group, st):
        """Worker body for one batch handed to `slot`.  A batch waits for
        memory only while it holds none (after giving back what it reserved),
        so that waiting batches never block each other: every holder is
        either running a pass or about to give its reservation back."""
        cv = st["cv"]
        dtype = group[0].A.dtype
        val_bytes = torch.tensor([], dtype=dtype).element_size()
        key = (slot, dtype)
        b = self._batch(slot, dtype)
        held = 0          # bytes this batch holds in st["used"] besides resident workspace
        counted = False   # this batch counts in st["inflight"]
        dropped = False   # the slot's plan was released once for this group

        def give_back():
            nonlocal held, counted
            st["used"] -= held
            held = 0
            if counted:
                st["inflight"] -= 1
                counted = False
            st["gen"] += 1
            cv.notify_all()

        def wait_for_release(gen0):
            # called with cv held and nothing reserved
            st["waits"] += 1
            cv.wait_for(lambda: st["gen"] != gen0 or st["inflight"] == 0 or st["errors"])

        try:
            with self._on_stream(self.streams[slot]):
                while True:
                    if st["errors"]:
                        return
                    As = [r.A for r in group]
                    Bs = [r.B for r in group]
                    rp_bytes = sum(A.rows + 1 for A in As) * self.idx_bytes
                    grow = max(0, b.workspace_query(As, Bs) - self.resident.get(key, 0))
                    pre = rp_bytes + grow
                    # (1) the symbolic pass's own allocations
                    with cv:
                        if st["used"] + pre > self.budget:
                            if len(group) > 1:
                                group = self._shrink(group, st)
                                continue
                            if st["inflight"] == 0:
                                if self.resident.get(key, 0) > 0:
                                    # this slot's own resident plan may be the obstacle
                                    b = self._drop_plan(slot, dtype)
                                    continue
                                self._reject(group[0], "symbolic footprint %d B exceeds the budget" % pre, st)
                                return
                            wait_for_release(st["gen"])
                            continue
                        st["used"] += pre
                        st["inflight"] += 1
                        counted = True
                        held = pre
                        st["peak"] = max(st["peak"], st["used"])
                    # (2) symbolic; the workspace actually grown stays resident
                    nnz = b.symbolic(As, Bs, fresh=True)
                    with cv:
                        actual = max(0, b.workspace_bytes - self.resident.get(key, 0))
                        self.resident[key] = max(self.resident.get(key, 0), b.workspace_bytes)
                        st["used"] -= grow - actual        # the query was an upper bound
                        held = rp_bytes
                    c_bytes = sum(z * (4 + val_bytes) for z in nnz)
                    # (3) C's columns and values
                    with cv:
                        if st["used"] + c_bytes <= self.budget:
                            st["used"] += c_bytes
                            held += c_bytes
                            st["peak"] = max(st["peak"], st["used"])
                            break
                        alone = st["inflight"] == 1
                        give_back()
                        if self.resident.get(key, 0) > self.keep_cap and not dropped:
                            # the plan's workspace may be what is in the way:
                            # release it and try once more with a fresh plan
                            b = self._drop_plan(slot, dtype)
                            dropped = True
                            continue
                        if len(group) == 1 and not alone:
                            wait_for_release(st["gen"])
                            continue
                    if len(group) > 1:
                        group = self._shrink(group, st)
                        dropped = False
                        continue
                    self._reject(group[0], "C of %d B does not fit the budget" % c_bytes, st)
                    return
                admitted = time.perf_counter() - st["t0"]
                outs = b.numeric(As, Bs)
                self.streams[slot].synchronize()
            done = time.perf_counter() - st["t0"]
            for r, C, z, pr in zip(group, outs, nnz, b.products):
                r.C = C if self.keep_results else None
                r.status = "ok"
                r.nnz = z
                r.products = pr
                r.admitted = admitted
                r.done = done
                r.batch_size = len(group)
            with cv:
                st["batch_sizes"].append(len(group))
        finally:
            # released also when a call above raised, so that no waiting slot
            # (and no join in run()) is left blocked
            with cv:
                give_back()
                if self.resident.get(key, 0) > self.keep_cap:
                    # a workspace grown this large by one batch is not kept
                    # for the next: release it
                    self._drop_plan(slot, dtype)

    def _drop_plan(self, slot, dtype):
        """Releases the slot's plan for `dtype` (called with the condition
        held, by the slot's own worker) and returns a fresh one."""
        key = (slot, dtype)
        b = self.batches[slot].pop(dtype, None)
        if b is not None:
            b.close()
        freed = self.resident.pop(key, 0)
        if self._st is not None:
            self._st["used"] -= freed
            self._st["gen"] += 1
            self._st["cv"].notify_all()
        return self._batch(slot, dtype)

    def _shrink(self, group, st):
        keep = max(1, len(group) // 2)
        with st["cv"]:
            st["shrinks"] += 1
            st["requeue"].extend(group[keep:])
        return group[:keep]

    def _worker(self, slot, tasks, st):
        while True:
            group = tasks.get()
            if group is None:
                return
            try:
                self._run_batch(slot, group, st)
            except BaseException as e:  # surfaced by run()
                with st["cv"]:
                    st["errors"].append(e)
                    st["cv"].notify_all()
            finally:
                st["idle"].put(slot)

    # -- scheduler -----------------------------------------------------------------
    def run(self, requests, poll_sleep: float = 5e-5) -> ServeStats:
        """Serves `requests` (released at their arrival times) and returns the
        statistics.  Every served request gets .C (if keep_results),
        .admitted, .done, .products, .nnz and status "ok"; a request that
        cannot fit the budget gets status "rejected" and .error.  An error
        raised by a worker is re-raised here once every worker has stopped."""
        pending = sorted(requests, key=lambda r: r.arrival)
        used0 = sum(self.resident.values())
        st = {"cv": threading.Condition(), "used": used0, "inflight": 0, "gen": 0, "peak": used0, "shrinks": 0,
              "waits": 0, "requeue": [], "batch_sizes": [], "errors": [], "rejected": [],
              "idle": _queue.Queue(), "t0": 0.0}
        self._st = st
        tasks = [_queue.Queue() for _ in range(self.nslots)]
        for s in range(self.nslots):
            st["idle"].put(s)
        workers = [threading.Thread(target=self._worker, args=(s, tasks[s], st), daemon=True)
                   for s in range(self.nslots)]
        for w in workers:
            w.start()
        waiting: list = []
        st["t0"] = time.perf_counter()
        pi = 0
        try:
            while True:
                with st["cv"]:
                    if st["errors"]:
                        raise st["errors"][0]
                    if st["requeue"]:
                        waiting[0:0] = st["requeue"]   # back to the head of the queue
                        waiting.sort(key=lambda r: r.arrival)
                        st["requeue"].clear()
                now = time.perf_counter() - st["t0"]
                while pi < len(pending) and pending[pi].arrival <= now:
                    waiting.append(pending[pi])
                    pi += 1
                if not waiting and pi >= len(pending) and st["idle"].qsize() == self.nslots:
                    with st["cv"]:
                        if not st["requeue"] and st["inflight"] == 0:
                            break
                dispatched = False
                while waiting:
                    try:
                        slot = st["idle"].get_nowait()
                    except _queue.Empty:
                        break
                    dtype = waiting[0].A.dtype
                    group = [r for r in waiting if r.A.dtype == dtype][: self.max_batch]
                    ids = {id(r) for r in group}
                    waiting = [r for r in waiting if id(r) not in ids]
                    tasks[slot].put(group)
                    dispatched = True
                if not dispatched:
                    time.sleep(poll_sleep)
        finally:
            for t in tasks:
                t.put(None)
            for w in workers:
                w.join()
        self._device_sync()
        served = [r for r in requests if r.status == "ok"]
        lat = sorted(r.latency for r in served) or [0.0]
        first = min(r.arrival for r in requests)
        last = max([r.done for r in requests if r.done is not None] or [first])
        span = max(last - first, 1e-9)
        prods = sum(r.products for r in served)
        per_kind = {}
        for r in served:
            per_kind.setdefault(r.kind or "job", []).append(r.latency)
        pk = {k: {"n": len(v), "p50_ms": round(1e3 * _pct(sorted(v), 0.5), 3),
                  "p99_ms": round(1e3 * _pct(sorted(v), 0.99), 3)} for k, v in per_kind.items()}
        bs = st["batch_sizes"]
        return ServeStats(
            requests=len(served), seconds=span, products=prods, gflops=2.0 * prods / span / 1e9,
            p50_ms=1e3 * _pct(lat, 0.5), p99_ms=1e3 * _pct(lat, 0.99),
            mean_batch=(sum(bs) / len(bs)) if bs else 0.0, batches=len(bs), peak_bytes=st["peak"],
            budget_bytes=self.budget, resymbolic=st["shrinks"], waits_for_memory=st["waits"],
            rejected=len(st["rejected"]), per_kind=pk)
