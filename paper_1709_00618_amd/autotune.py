"""Autotuner of the launch schedule of the batched tracker.

The knobs (``tpcca_tuning_t``) change occupancy, load balance and grid
granularity, never a result: every decision compares cluster IDs and each
tracklet sees the same operation sequence whatever the schedule.  The tuner
replays the batch graph of a sample batch and searches the knobs one at a
time (coordinate descent from the default schedule: each knob's values are
timed with the others at their best so far, in the order of ``SPACE``, for
``rounds`` passes), keeps the fastest point, and caches it in
``tuning_cache.json`` keyed by device name and a size bucket of the batch
(clusters, units).  Given a second context, a point is timed with two
batches in flight (the contexts fed alternately), the way the batched bench
and the server run: then the cost per batch includes how well one batch's
stages fill the other's fit drain.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning_cache.json")

# knob -> values; the first value is the default schedule's
SPACE = {
    "fit_block": [0, 64, 256],
    "fit_blocks_per_cu": [0, 6, 4, 8, 12],
    "fit_min_waves": [0, 4],
    "fit_pool": [64, 128, 32],
    "link_stage": [0, 1, 2],
    "link_tile": [0, 128, 512],
}
DEFAULT = {k: v[0] for k, v in SPACE.items()}


def bucket(n_clusters: int, n_units: int) -> str:
    return f"cl2^{max(0, int(math.log2(max(1, n_clusters))))}_u{'1' if n_units <= 1 else '36' if n_units <= 36 else 'many'}"


def device_name() -> str:
    """Cache key of the device: its GPU architecture (the marketing name can
    differ between environments on the same hardware)."""
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # plumbing only
        return "unknown"


def load_cache() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def lookup(n_clusters: int, n_units: int, dev: str | None = None):
    return load_cache().get(dev or device_name(), {}).get(bucket(n_clusters, n_units))


def store(entry: dict, n_clusters: int, n_units: int, dev: str | None = None, path: str = CACHE):
    cache = load_cache()
    cache.setdefault(dev or device_name(), {})[bucket(n_clusters, n_units)] = entry
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def _time(ctx, run, reps):
    run()
    ctx.sync()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        run()
        ctx.sync()
        ts.append(time.perf_counter() - t0)
    ts.sort()
    return ts[len(ts) // 2]


def _time_pipelined(ctxs, run, frames=8, reps=2):
    """Median over reps of the time per batch with len(ctxs) batches in flight."""
    for i in range(2 * len(ctxs)):
        run(ctxs[i % len(ctxs)])
    for c in ctxs:
        c.sync()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        for i in range(frames):
            run(ctxs[i % len(ctxs)])
        for c in ctxs:
            c.sync()
        ts.append((time.perf_counter() - t0) / frames)
    ts.sort()
    return ts[len(ts) // 2]


def tune(ctx, cl, row, units, device=True, reps=3, space=None, log=None, ctx2=None, rounds=1):
    """Coordinate search of the schedule on one batch; returns (best dict,
    table of (seconds, knobs) for every point timed).  With ctx2, every
    point is timed with two batches in flight."""
    space = space or SPACE
    ctxs = [ctx] if ctx2 is None else [ctx, ctx2]
    seen = {}

    def run(c=ctx):
        c.run_batch(cl, row, units, device=device, graph=True)

    def timed(knobs):
        key = tuple(sorted(knobs.items()))
        if key not in seen:
            for c in ctxs:
                c.reset()
                c.set_tuning(**knobs)
            seen[key] = _time(ctx, run, reps) if ctx2 is None else _time_pipelined(ctxs, run)
            if log:
                log(f"autotune {knobs}: {seen[key] * 1e3:.3f} ms")
        return seen[key]

    best = {k: v[0] for k, v in space.items()}
    best_t = timed(best)
    for _ in range(rounds):
        for name, vals in space.items():
            for v in vals:
                point = dict(best, **{name: v})
                t = timed(point)
                if t < best_t:
                    best, best_t = point, t
    table = sorted(((t, dict(k)) for k, t in seen.items()), key=lambda x: x[0])
    for c in ctxs:
        c.reset()
        c.set_tuning(**best)
    return best, table


def tuned(ctx, cl, row, units, n_clusters, device=True, log=None, retune=False, ctx2=None):
    """Apply the cached schedule for this device and size, tuning first if
    there is none (with ctx2: timed with two batches in flight).  Returns
    (knobs, source)."""
    n_units = len(units)
    entry = None if retune else lookup(n_clusters, n_units)
    if entry is not None:
        for c in [ctx] if ctx2 is None else [ctx, ctx2]:
            c.reset()
            c.set_tuning(**entry["knobs"])
        return entry["knobs"], "cache"
    best, table = tune(ctx, cl, row, units, device=device, log=log, ctx2=ctx2)
    store({"knobs": best, "ms": round(table[0][0] * 1e3, 4), "in_flight": 1 if ctx2 is None else 2,
           "default_ms": round(next(t for t, k in table if k == _default(table)) * 1e3, 4)
           if _default(table) else None},
          n_clusters, n_units)
    return best, "tuned"


def _default(table):
    return DEFAULT if any(k == DEFAULT for _, k in table) else None
