"""Serving loop for SpGEMM requests with continuous batching.

Requests (operands already in device memory) arrive over time.  The
scheduler thread moves arrived requests to a queue and, whenever a slot is
idle, hands it a batch: the oldest waiting request and the following ones
with the same value type, up to `max_batch`.  Each slot owns a stream, one
plan per value type and a host worker thread, which
  1. runs the batched symbolic pass (blocking only its own thread: the C
     calls release the interpreter lock, and the wait is on its own stream),
  2. computes the batch's exact footprint -- C's columns, values and row
     pointers plus the plan's workspace -- and admits the batch if it fits
     the HBM budget next to what is in flight; otherwise it gives the newest
     half of the batch back to the queue and retries with the rest, and a
     single request that does not fit waits until memory is released (or
     runs at once if nothing else is in flight),
  3. enqueues the numeric pass, waits for its own stream, stamps every
     request of the batch with its completion time and releases the memory.
Batches on different slots overlap on the device and on the host, and
requests that arrive while others run are batched into the next free slot.
Latency is arrival to the completion of the request's batch on the device,
as seen by the host."""
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
    requests: int
    seconds: float                    # first arrival to last completion
    products: int
    gflops: float
    p50_ms: float
    p99_ms: float
    mean_batch: float
    batches: int
    peak_bytes: int
    resymbolic: int                   # batches shrunk to fit the budget
    waits_for_memory: int
    per_kind: dict = field(default_factory=dict)


def _pct(sorted_vals, q):
    return sorted_vals[min(len(sorted_vals) - 1, int(q * len(sorted_vals)))]


class Server:
    # Two slots overlap one batch's host work and symbolic pass with another's
    # numeric pass.  Measured on an MI355X with the served job mix at 0.8x of
    # the closed-loop rate: one or two slots keep up (two: p50 82 ms, p99
    # 0.4 s), four fall behind (p50 2 s).
    def __init__(self, slots: int = 2, hbm_budget_bytes: float = 64e9, max_batch: int = 16,
                 keep_results: bool = True, c_index_dtype=torch.int64, **options):
        self.nslots = slots
        self.budget = int(hbm_budget_bytes)
        self.max_batch = max_batch
        self.keep_results = keep_results
        self.c_index_dtype = c_index_dtype
        self.options = options
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.batches = [dict() for _ in range(slots)]   # value dtype -> Batch on that slot's stream
        self.idx_bytes = torch.tensor([], dtype=c_index_dtype).element_size()

    def close(self):
        for d in self.batches:
            for b in d.values():
                b.close()
        self.batches = [dict() for _ in range(self.nslots)]

    # -- worker side -------------------------------------------------------------
    def _batch(self, slot, dtype) -> Batch:
        b = self.batches[slot].get(dtype)
        if b is None:
            b = Batch(dtype, self.c_index_dtype, stream=self.streams[slot], **self.options)
            self.batches[slot][dtype] = b
        return b

    def _run_batch(self, slot, group, st):
        """Worker body for one batch handed to `slot`."""
        dtype = group[0].A.dtype
        val_bytes = torch.tensor([], dtype=dtype).element_size()
        b = self._batch(slot, dtype)
        with torch.cuda.stream(self.streams[slot]):
            while True:
                As = [r.A for r in group]
                Bs = [r.B for r in group]
                nnz = b.symbolic(As, Bs, fresh=True)
                need = sum(z * (4 + val_bytes) for z in nnz) + sum(A.rows + 1 for A in As) * self.idx_bytes
                need += b.workspace_bytes
                with st["cv"]:
                    if st["in_use"] + need <= self.budget or st["inflight"] == 0:
                        st["in_use"] += need
                        st["inflight"] += 1
                        st["peak"] = max(st["peak"], st["in_use"])
                        break
                    if len(group) > 1:
                        keep = max(1, len(group) // 2)
                        back = group[keep:]
                        group = group[:keep]
                        st["shrinks"] += 1
                        st["requeue"].extend(back)
                        continue
                    st["waits"] += 1
                    st["cv"].wait_for(lambda: st["in_use"] + need <= self.budget or st["inflight"] == 0)
                    st["in_use"] += need
                    st["inflight"] += 1
                    st["peak"] = max(st["peak"], st["in_use"])
                    break
            admitted = time.perf_counter() - st["t0"]
            outs = b.numeric(As, Bs)
            self.streams[slot].synchronize()
        done = time.perf_counter() - st["t0"]
        for r, C, z, pr in zip(group, outs, nnz, b.products):
            r.C = C if self.keep_results else None
            r.nnz = z
            r.products = pr
            r.admitted = admitted
            r.done = done
            r.batch_size = len(group)
        with st["cv"]:
            st["in_use"] -= need
            st["inflight"] -= 1
            st["batch_sizes"].append(len(group))
            st["cv"].notify_all()

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
        statistics.  Every request gets .C (if keep_results), .admitted,
        .done, .products, .nnz."""
        pending = sorted(requests, key=lambda r: r.arrival)
        st = {"cv": threading.Condition(), "in_use": 0, "inflight": 0, "peak": 0, "shrinks": 0, "waits": 0,
              "requeue": [], "batch_sizes": [], "errors": [], "idle": _queue.Queue(), "t0": 0.0}
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
        torch.cuda.synchronize()
        lat = sorted(r.latency for r in requests)
        first = min(r.arrival for r in requests)
        last = max(r.done for r in requests)
        span = max(last - first, 1e-9)
        prods = sum(r.products for r in requests)
        per_kind = {}
        for r in requests:
            per_kind.setdefault(r.kind or "job", []).append(r.latency)
        pk = {k: {"n": len(v), "p50_ms": round(1e3 * _pct(sorted(v), 0.5), 3),
                  "p99_ms": round(1e3 * _pct(sorted(v), 0.99), 3)} for k, v in per_kind.items()}
        bs = st["batch_sizes"]
        return ServeStats(
            requests=len(requests), seconds=span, products=prods, gflops=2.0 * prods / span / 1e9,
            p50_ms=1e3 * _pct(lat, 0.5), p99_ms=1e3 * _pct(lat, 0.99),
            mean_batch=(sum(bs) / len(bs)) if bs else 0.0, batches=len(bs), peak_bytes=st["peak"],
            resymbolic=st["shrinks"], waits_for_memory=st["waits"], per_kind=pk)
