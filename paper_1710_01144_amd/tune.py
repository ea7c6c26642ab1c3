"""Autotuners: the engine's launch shapes (gc_tuning) and the lazy loop's
batch schedule (block, growth).

The shapes -- adjacency entries per thread per step, entries per workgroup
before a level takes more workgroups, workgroups per CU of a level kernel --
decide only how a gain or update launch is spread over the GPU; groups,
farness, gains and evaluation counts are the same for every choice.  The
tuner times whole greedy jobs on the graph at hand, changing one shape at a
time from the current setting (one pass of coordinate descent over a small
grid), keeps the fastest and caches it per graph signature and job in a JSON
file.

The batch schedule -- candidates per launch at the start of a round (block)
and the factor by which each further launch of the round grows (growth) --
changes how many candidates are evaluated and in how many launches, never a
pick: every candidate whose stale gain can still beat the best of the
launches before is evaluated, whatever the schedule.  autotune_schedule times
whole jobs over a small grid of (block, growth), checks that every schedule
returns the same group, and keeps the fastest.
"""
from __future__ import annotations

import json
import os

GRID = {
    "unroll": (4, 8, 16),
    "unroll_small": (4, 8),
    "min_edges": (256, 512, 1024, 2048),
    "min_edges_small": (128, 256, 512, 1024),
    "level_wgs_per_cu": (2, 4, 8),
}


def signature(G) -> str:
    """Graph signature for the cache: size, degree spread and a row-pointer digest."""
    import hashlib
    import numpy as np
    rp = G.row_ptr.cpu().numpy() if hasattr(G.row_ptr, "cpu") else np.asarray(G.row_ptr)
    deg = np.diff(rp.astype(np.int64))
    h = hashlib.sha256(rp.astype(np.int32).tobytes()).hexdigest()[:12]
    return "n%d-nnz%d-maxdeg%d-%s" % (len(rp) - 1, int(rp[-1]), int(deg.max(initial=0)), h)


def job_key(sig: str, k: int, order: str, block: int) -> str:
    return "%s|k%d|%s|b%d" % (sig, k, order, block)


def load_cache(path: str) -> dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save_cache(path: str, cache: dict) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_job(G, k, order, block, reps, mlp_params=None) -> float:
    """Best host wall time (ms) of `reps` greedy jobs after one warm-up."""
    G.greedy_group(k, order=order, block=block, mlp_params=mlp_params)
    best = float("inf")
    for _ in range(reps):
        _, _, st = G.greedy_group(k, order=order, block=block, mlp_params=mlp_params)
        best = min(best, float(st["ms_total"]))
    return best


def autotune(G, k: int, order: str = "plain", block: int = 64, reps: int = 2, cache_path: str = None,
             grid: dict = None, mlp_params=None) -> dict:
    """Pick the fastest launch shapes for greedy jobs of this size on G and
    leave them set on G.  With a cache file that already holds this graph and
    job, its entry is applied without timing.  Returns
    {"shape", "ms_default", "ms_tuned", "trials", "cached"}."""
    grid = grid or GRID
    cache_path = cache_path or os.environ.get("GC_TUNE_CACHE")
    key = job_key(signature(G), k, order, block)
    cache = load_cache(cache_path)
    if key in cache:
        G.set_tuning(**cache[key]["shape"])
        return dict(cache[key], cached=True)
    shape = G.get_tuning()
    ms0 = _time_job(G, k, order, block, reps, mlp_params)
    best_ms, trials = ms0, 1
    for field, values in grid.items():
        start = shape[field]
        for v in values:
            if v == start:
                continue
            G.set_tuning(**dict(shape, **{field: v}))
            ms = _time_job(G, k, order, block, reps, mlp_params)
            trials += 1
            if ms < best_ms:
                best_ms, shape = ms, dict(shape, **{field: v})
        G.set_tuning(**shape)
    out = {"shape": shape, "ms_default": round(ms0, 3), "ms_tuned": round(best_ms, 3), "trials": trials}
    if cache_path:
        cache[key] = out
        save_cache(cache_path, cache)
    return dict(out, cached=False)


SCHEDULES = [(b, gr) for b in (32, 64, 128, 256) for gr in (1, 2, 4, 8)]


def autotune_schedule(G, k: int, order: str = "plain", schedules=None, reps: int = 2,
                      cache_path: str = None, mlp_params=None) -> dict:
    """The fastest (block, growth) for greedy jobs of this size on G.  Every
    schedule must give the same group and farness (AssertionError otherwise).
    Returns {"block", "growth", "ms", "ms_default", "table", "cached"}; the
    default is (64, 2)."""
    schedules = schedules or SCHEDULES
    cache_path = cache_path or os.environ.get("GC_TUNE_CACHE")
    key = "%s|k%d|%s|schedule" % (signature(G), k, order)
    cache = load_cache(cache_path)
    if key in cache:
        return dict(cache[key], cached=True)
    ref = None
    table = {}
    for blk, gr in schedules:
        grp, far, _ = G.greedy_group(k, order=order, block=blk, block_growth=gr, mlp_params=mlp_params)
        got = (list(map(int, grp)), list(map(int, far))) if grp is not None else None
        if ref is None:
            ref = got
        assert got == ref, "schedule (%d, %d) changed the picks" % (blk, gr)
        best = float("inf")
        for _ in range(reps):
            _, _, st = G.greedy_group(k, order=order, block=blk, block_growth=gr, mlp_params=mlp_params)
            best = min(best, float(st["ms_total"]))
        table["%d,%d" % (blk, gr)] = round(best, 3)
    pick = min(table, key=lambda kk: (table[kk], kk))
    blk, gr = (int(x) for x in pick.split(","))
    out = {"block": blk, "growth": gr, "ms": table[pick], "ms_default": table.get("64,2"), "table": table}
    if cache_path:
        cache[key] = out
        save_cache(cache_path, cache)
    return dict(out, cached=False)
