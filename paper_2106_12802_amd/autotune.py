"""Autotuner of the renderer's launch shape (performance only: results are bitwise
independent of the tuning, which the tests check).

It times a workload under each candidate (chunk_paths, trace_blocks, schedule), keeps the
fastest, and caches the choice in a JSON file keyed by device and workload so that
later runs apply it without measuring.
"""
from __future__ import annotations

import json
import os
import time

from . import tracer as T

CHUNKS = (1 << 21, 1 << 22, 1 << 23, 1 << 24, 1 << 25)
BLOCKS = (512, 1024, 2048, 4096)
SCHEDULES = (0, 1)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mrs_autotune.json")


def _device_key():
    import torch
    p = torch.cuda.get_device_properties(0)
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}"


def choose(timings):
    """The candidate with the smallest median time; ties go to the earlier candidate."""
    best = None
    for cand, times in timings:
        ts = sorted(times)
        med = ts[len(ts) // 2]
        if best is None or med < best[1]:
            best = (cand, med)
    return best


def tune(workload, key, cache_path=DEFAULT_CACHE, reps=3, candidates=None, log=None,
         force=False):
    """Pick and apply the fastest tuning for `workload` (a callable that enqueues the
    renders); returns {"chunk_paths", "trace_blocks", "schedule", "ms", "cached"}."""
    import torch
    full_key = f"{_device_key()}|{key}"
    cache = {}
    if os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if not force and full_key in cache:
        c = cache[full_key]
        T.set_tuning(c["chunk_paths"], c["trace_blocks"], c["schedule"])
        return dict(c, cached=True)
    if candidates is None:
        candidates = [(c, b, s) for c in CHUNKS for b in BLOCKS for s in SCHEDULES]
    timings = []
    for chunk, blocks, sched in candidates:
        T.set_tuning(chunk, blocks, sched)
        workload()  # warm-up: grows buffers outside the timing
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            workload()
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        timings.append(((chunk, blocks, sched), times))
        if log:
            log(f"[autotune] chunk {chunk} blocks {blocks} schedule {sched}: "
                f"{sorted(times)[len(times) // 2]:.3f} ms")
    (chunk, blocks, sched), ms = choose(timings)
    T.set_tuning(chunk, blocks, sched)
    cache[full_key] = {"chunk_paths": chunk, "trace_blocks": blocks, "schedule": sched,
                       "ms": round(ms, 4)}
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path + ".tmp", "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(cache_path + ".tmp", cache_path)
    except OSError:
        pass
    return dict(cache[full_key], cached=False)
