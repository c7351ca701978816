"""Autotuner for batched products: times candidate launch parameters (bin
thresholds, hash-table admission, long-row column segment, workgroups per CU
of the long-row symbolic pass) on a sample of the batch and keeps the fastest per
workload signature in a JSON cache.  Every candidate computes the same result
(thresholds only decide which kernel handles a row); the tuner measures, it
never changes the arithmetic."""
from __future__ import annotations

import json
import os
import time

import torch

from . import Batch

# Candidate option sets (reap_options_t fields).  The first is the library's
# default configuration.
CANDIDATES = (
    {},
    {"wave_max_products": 512},
    {"wave_max_products": -1},
    {"wave_small_values": 64},
    {"wave_hash_products": -1},
    {"group_lds_span": 65536},
    {"long_workgroups_per_cu": 1},
    {"long_workgroups_per_cu": 4},
    {"wave_max_products": -1, "long_workgroups_per_cu": 4},
)


def default_cache_path() -> str:
    base = os.environ.get("REAP_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "reap_spgemm")
    return base if base.endswith(".json") else os.path.join(base, "autotune.json")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_batch(As, Bs, dtype, options, reps=2, stream=None) -> float:
    """Median wall-clock seconds of symbolic + numeric for the batch (graph
    replays after one warm-up call), device work included."""
    times = []
    with Batch(dtype, graph=True, stream=stream, **options) as b:
        for r in range(reps + 1):
            b.synchronize()
            t0 = time.perf_counter()
            b.symbolic(As, Bs)
            b.numeric(As, Bs)
            b.synchronize()
            if r > 0:
                times.append(time.perf_counter() - t0)
    times.sort()
    return times[len(times) // 2]


# Results measured on an MI355X, shipped with the package and consulted when
# the user cache has no entry for a signature.
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def lookup(signature: str, cache_path: str | None = None):
    """Cached entry for `signature` (user cache first, then the shipped one), or None."""
    for path in (cache_path or default_cache_path(), SHIPPED):
        entry = _load(path).get(signature)
        if entry:
            return entry
    return None


def tune(As, Bs, dtype, signature: str, cache_path: str | None = None, reps: int = 2,
         candidates=CANDIDATES, force: bool = False) -> dict:
    """Options for this workload: from a cache when `signature` is there
    (unless `force`), else measured over `candidates` on (As, Bs) and written
    to the user cache.  Returns {"options": ..., "seconds": ..., "trials": [...]}."""
    path = cache_path or default_cache_path()
    if not force:
        entry = lookup(signature, path)
        if entry:
            return entry
    cache = _load(path)
    trials = []
    for opts in candidates:
        s = time_batch(As, Bs, dtype, opts, reps=reps)
        trials.append({"options": dict(opts), "seconds": s})
    best = min(trials, key=lambda t: t["seconds"])
    entry = {"options": best["options"], "seconds": best["seconds"], "trials": trials,
             "device": torch.cuda.get_device_name(0) if torch.cuda.is_available() else "",
             "products": len(As)}
    cache[signature] = entry
    _save(path, cache)
    return entry
