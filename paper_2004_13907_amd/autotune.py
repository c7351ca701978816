"""Autotuner for batched products: searches launch parameters -- bin
thresholds, which rows take the medium (256-thread) long-row workgroups, the
shape and count of the symbolic long-row workgroups, the long-row LDS
accumulator -- on a sample of the batch and keeps the fastest per workload
signature in a JSON cache.  Every setting computes the same result
(thresholds and shapes only decide which kernel and workgroup handle a row);
the tuner measures, it never changes the arithmetic.

The search is a coordinate descent over SPACE: starting from the library's
defaults, each dimension in turn is set to each of its values with the
others held at the best found so far, and the fastest is kept; passes repeat
until one changes nothing (or `max_passes`).  Settings already timed are not
timed again."""
from __future__ import annotations

import json
import os
import time

import torch

from . import Batch

# Search space: one reap_options_t field per dimension and the values it may
# take; the first value of each is the library default (0).
SPACE = (
    ("wave_max_products", (0, 512, -1)),      # wavefront rows: up to 1024 products, 512, or none
    ("wave_small_values", (0, 64)),           # compact wavefront rows: up to 128 entries of C, or 64
    ("wave_hash_products", (0, -1)),          # wavefront hash rows: up to half the table's slots, or none
    ("wave_hash_slots", (0, 1024)),           # wavefront hash table: 512 slots, or 1024 (rows up to 512 products)
    ("mid_values", (0, 1024, -1)),            # medium long-row workgroups: rows up to 2048 entries, 1024, none
    ("long_sym_narrow", (0, -1)),             # symbolic long-row workgroups: 256 threads when possible, or 512
    ("long_workgroups_per_cu", (0, 1, 4)),    # symbolic long-row workgroups per CU: 2 (x2 narrow), 1, 4
    ("group_lds_values", (0, 4096)),          # large long-row LDS accumulator: 8192 slots, or 4096
)


def default_cache_path() -> str:
    base = os.environ.get("REAP_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "reap_spgemm")
    return base if base.endswith(".json") else os.path.join(base, "autotune.json")


def _load(path):
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
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


def _options(point) -> dict:
    """reap_options_t fields of a point of the space (defaults left out)."""
    return {k: v for k, v in point.items() if v != 0}


def search(measure, space=SPACE, max_passes: int = 3):
    """Coordinate descent over `space`; `measure(options)` returns seconds.
    Returns (best options, best seconds, trials in the order timed)."""
    point = {k: vals[0] for k, vals in space}
    seen = {}
    trials = []

    def cost(pt):
        key = tuple(sorted(_options(pt).items()))
        if key not in seen:
            s = float(measure(_options(pt)))
            seen[key] = s
            trials.append({"options": _options(pt), "seconds": s})
        return seen[key]

    best = cost(point)
    for _ in range(max_passes):
        changed = False
        for name, vals in space:
            for v in vals:
                if v == point[name]:
                    continue
                cand = dict(point)
                cand[name] = v
                s = cost(cand)
                if s < best:
                    best, point, changed = s, cand, True
        if not changed:
            break
    return _options(point), best, trials


def tune(As, Bs, dtype, signature: str, cache_path: str | None = None, reps: int = 2, space=SPACE,
         force: bool = False, max_passes: int = 3) -> dict:
    """Options for this workload: from a cache when `signature` is there
    (unless `force`), else searched over `space` on (As, Bs) and written to
    the user cache.  Returns {"options": ..., "seconds": ..., "trials": [...]}."""
    path = cache_path or default_cache_path()
    if not force:
        entry = lookup(signature, path)
        if entry:
            return entry
    opts, secs, trials = search(lambda o: time_batch(As, Bs, dtype, o, reps=reps), space, max_passes)
    entry = {"options": opts, "seconds": secs, "trials": trials,
             "device": torch.cuda.get_device_name(0) if torch.cuda.is_available() else "",
             "products": len(As), "search": "coordinate descent over %d dimensions" % len(space)}
    cache = _load(path)
    cache[signature] = entry
    _save(path, cache)
    return entry
