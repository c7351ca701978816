#!/usr/bin/env python3
"""SpGEMM benchmark on one MI355X.

A step is one pass of the whole product path over one synthetic input:
symbolic (row product counts, binning, per-row column counts, scan, nnz(C) to
the host), allocation of C, and numeric.  Inputs are resident in device memory
before the timed region.  The default workload is C = A*A for the 27-point
stencil on a 64^3 grid in FP64 (262,144 rows).

Prints one JSON line: GFLOP/s = 2 x partial products per second, the roofline
figure of the dominant kernel (device time from HIP events recorded by the
library on its stream during the timed steps), and the oracle timed on the
host cores as the CPU baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0           # MI355X HBM3E, published peak
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["paper_2004_13907_amd/csrc/kernels_numeric.h", "paper_2004_13907_amd/csrc/kernels_symbolic.h",
                  "paper_2004_13907_amd/csrc/device_utils.h", "paper_2004_13907_amd/csrc/spgemm_common.h"]

WORKLOADS = {
    "stencil": "stencil27 64^3: C = A*A, 262144 rows, FP64, CSR int32",
    "uniform": "uniform 2000x2000, 10 nnz/row: C = A*A, FP64, CSR int32",
    "rmat": "R-MAT scale 18 (a,b,c,d = .57,.19,.19,.05), edge factor 16: C = A*A^T, FP32, CSR int32",
}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def csr_bytes(rows, nnz, idx_bytes, val_bytes) -> int:
    """Bytes of one CSR matrix as stored: row pointer + column indices + values."""
    return (rows + 1) * idx_bytes + nnz * (4 + val_bytes)


def make_workload(name):
    import numpy as np
    import synth
    if name == "stencil":
        A = synth.stencil27(64, seed=2)
        return A, A, np.float64
    if name == "uniform":
        A = synth.uniform_rows(2000, 2000, 10, seed=1)
        return A, A, np.float64
    if name == "rmat":
        A = synth.rmat(18, seed=3)
        return A, synth.transpose(A), np.float32
    raise ValueError(name)


def read_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources; otherwise None."""
    path = os.path.join(PROFILES, "traffic_%s_%s.txt" % (kernel, workload))
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(A, B, products, budget_s: float):
    """The oracle (never tuned) on the host cores, on the whole workload,
    repeated until about budget_s seconds of work; median time."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    threads = max(1, min(cores, oracle.max_threads() if os.environ.get("OMP_NUM_THREADS") else cores))
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        oracle.spgemm(A, B, threads=threads)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > budget_s or len(times) >= 50:
            break
    times.sort()
    med = times[len(times) // 2]
    return {"value": round(2.0 * products / med / 1e9, 4), "unit": "GFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": "whole workload (all rows), %d repetitions, median %.3f s" % (len(times), med)}


def calib_copy(gib: float = 1.0, reps: int = 5):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = int(gib * (1 << 30)) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes_read": n * 8, "calib_copy_bytes_written": n * 8, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="stencil", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true", help="only run the counter-calibration copy")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d, WORLD_SIZE %d requested)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2004_13907_amd as reap

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.calib_copy:
        calib_copy()
        return

    A, B, npdt = make_workload(args.workload)
    tdt = torch.float64 if npdt == np.float64 else torch.float32
    dA = reap.DeviceCSR.from_host(A, dtype=tdt)
    dB = dA if B is A else reap.DeviceCSR.from_host(B, dtype=tdt)
    plan = reap.Plan(tdt, torch.int32, profile=1)
    rp = torch.empty(A.rows + 1, dtype=torch.int32, device="cuda")

    stamps = []

    def step():
        _, nnz, prods = plan.symbolic(dA, dB, rp)
        stamps.append(time.perf_counter())
        col = torch.empty(nnz, dtype=torch.int32, device="cuda")
        val = torch.empty(nnz, dtype=tdt, device="cuda")
        plan.numeric(dA, dB, rp, col, val)
        return nnz, prods

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.phase_reset()
    stamps.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        nnz, prods = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    phases = plan.phase_times()
    bins = plan.bin_stats()

    ms_step = elapsed / args.steps * 1e3
    gflops = 2.0 * prods * args.steps / elapsed / 1e9
    val_bytes = 8 if tdt == torch.float64 else 4
    alg_bytes = csr_bytes(A.rows, A.nnz, 4, val_bytes) + csr_bytes(B.rows, B.nnz, 4, val_bytes) + \
        csr_bytes(A.rows, nnz, 4, val_bytes)
    # per-step latency from successive symbolic completions (steady state)
    lat = np.diff(np.array(stamps)) * 1e3 if len(stamps) > 1 else np.array([ms_step])

    # dominant kernel by measured device time
    kern = {
        "k_num_wave_bmp": phases["numeric_wave_bitmap"],
        "k_num_wave_hash": phases["numeric_wave_hash"],
        "k_num_group": phases["numeric_group"],
        "k_sym_wave+k_sym_group": phases["symbolic"],
    }
    dom = max(kern, key=kern.get)
    dom_ms = kern[dom]
    if dom.startswith("k_sym"):
        # symbolic: A pattern + B pattern read, per-row class/count/window written
        dom_bytes = (A.rows + 1) * 4 + A.nnz * 4 + (B.rows + 1) * 4 + B.nnz * 4 + A.rows * 13
    else:
        dom_bytes = alg_bytes
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else 0.0
    traffic = read_traffic(dom.split("+")[0], args.workload)

    out = {
        "metric": "SpGEMM GFLOP/s (2 x partial products per second)",
        "value": round(gflops, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if tdt == torch.float64 else "f32 (f64 accumulate)",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "rows": A.rows, "nnz_A": A.nnz, "nnz_B": B.nnz,
                   "products": prods, "nnz_C": nnz},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic, "kernel_ms": round(dom_ms, 5),
                     "algorithmic_bytes_per_launch": dom_bytes},
        "step_algorithmic_GBps": round(alg_bytes / (ms_step * 1e-3) / 1e9, 1),
        "step_hbm_frac": round(alg_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4), "p99": round(float(np.percentile(lat, 99)), 4)},
        "phases_ms": {k: round(v, 5) for k, v in phases.items() if k != "calls"},
        "bins": bins,
        "source_hash": kernel_source_hash(),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, B, prods, args.cpu_seconds)
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
