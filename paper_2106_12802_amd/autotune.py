"""Autotuner of the renderer's and the network's launch shape (performance only:
results are bitwise independent of the tuning, which the tests check).

It times a workload under candidate tunings, keeps the fastest, and caches the
choice in a JSON file keyed by device and workload so that later runs apply it
without measuring.  The search is a grid over the primary launch shape
(resident paths x traversal grid x queue schedule) followed by one pass over
each secondary knob with the rest held at the best so far: sub-chunk streams,
the first bounce traced path by path, the ordering of appended rays, the BVH
node format, the bounces traced a wave at a time, the network conv tile plan
and the fused residual blocks.
"""
from __future__ import annotations

import json
import os
import time

from . import tracer as T

CHUNKS = (1 << 21, 1 << 22, 1 << 23, 1 << 24, 1 << 25)
BLOCKS = (1024, 2048, 4096, 8192)
SCHEDULES = (0, 1)
SECONDARY = (("streams", (1, 2, 3, 4)), ("tail_bounce", (2, 3, 4, 5)),
             ("queue_sort", (0, 1)), ("bvh_quantized", (0, 1)),
             ("wave_extend", (0, 1, 2)), ("wave_shadow", (0, 1, 2)),
             ("conv_small_tiles", (0, 64, 128, 256)), ("net_fused_blocks", (0, 1)))
KEYS = ("chunk_paths", "trace_blocks", "schedule", "streams", "tail_bounce", "queue_sort",
        "bvh_quantized", "wave_extend", "wave_shadow", "conv_small_tiles", "net_fused_blocks")
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


def as_dict(cand):
    """A candidate as a tuning dict: a (chunk_paths, trace_blocks, schedule) tuple or a dict."""
    if isinstance(cand, dict):
        return dict(cand)
    return dict(zip(("chunk_paths", "trace_blocks", "schedule"), cand))


def _apply(base, cand):
    t = dict(base)
    t.update(as_dict(cand))
    T.set_tuning(**{k: t[k] for k in T.TUNING_KEYS})
    return t


def tune(workload, key, cache_path=DEFAULT_CACHE, reps=3, candidates=None, log=None,
         force=False, secondary=None):
    """Pick and apply the fastest tuning for `workload` (a callable that enqueues the
    work); returns the chosen tuning fields plus "ms" and "cached".

    candidates: the primary grid (tuples or dicts; default CHUNKS x BLOCKS x
    SCHEDULES); secondary: [(field, values)] searched one field at a time after
    it (default SECONDARY; [] to skip)."""
    import torch
    full_key = f"{_device_key()}|{key}"
    cache = {}
    if os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    base = T.get_tuning()
    if not force and full_key in cache:
        c = cache[full_key]
        _apply(base, {k: c[k] for k in KEYS if k in c})
        return dict(c, cached=True)
    if candidates is None:
        candidates = [(c, b, s) for c in CHUNKS for b in BLOCKS for s in SCHEDULES]
    if secondary is None:
        secondary = SECONDARY

    def measure(cands, cur):
        timings = []
        for cand in cands:
            t = _apply(cur, cand)
            workload()  # warm-up: grows buffers outside the timing
            torch.cuda.synchronize()
            times = []
            for _ in range(reps):
                t0 = time.perf_counter()
                workload()
                torch.cuda.synchronize()
                times.append((time.perf_counter() - t0) * 1e3)
            timings.append((as_dict(cand), times))
            if log:
                shown = {k: t[k] for k in KEYS}
                log(f"[autotune] {shown}: {sorted(times)[len(times) // 2]:.3f} ms")
        return choose(timings)

    best, ms = measure(candidates, base)
    cur = dict(base)
    cur.update(best)
    for field, values in secondary:
        b, m = measure([{field: v} for v in values], cur)
        if m < ms:
            cur.update(b)
            ms = m
    _apply(base, cur)
    chosen = {k: int(cur[k]) for k in KEYS}
    cache[full_key] = dict(chosen, ms=round(ms, 4))
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path + ".tmp", "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(cache_path + ".tmp", cache_path)
    except OSError:
        pass
    return dict(cache[full_key], cached=False)
