"""Tile autotuner: times a few candidate work decompositions
(sip_batch_set_tiles) on the batch that will run, and keeps the fastest per
workload class (field type, dimensionality, total-size class, instance
count class) in a JSON cache.

Results are bit-reproducible for a fixed tile setting; a different setting
changes the summation order of the per-item partial sums (not the math)."""
from __future__ import annotations

import json
import math
import os

CANDIDATES = [
    # (pt_points, pt_max_items, thr_points, thr_max_items, pt_threads, cg_form)
    (2048, 512, 2048, 512, 512, 0),
    (1024, 512, 2048, 512, 512, 0),
    (2048, 1024, 4096, 512, 512, 0),
    (4096, 512, 4096, 256, 512, 0),
    (4096, 1024, 8192, 512, 512, 0),
    (1024, 1024, 2048, 512, 256, 0),
    (2048, 512, 2048, 512, 256, 0),
    (2048, 1024, 4096, 512, 256, 0),
    (4096, 512, 4096, 256, 256, 0),
    (1024, 2048, 2048, 512, 256, 0),
    # large grids: threshold items of four full block rounds (4096 float points)
    (1024, 512, 2048, 1024, 512, 0),
    (2048, 512, 2048, 1024, 512, 0),
    # one launch per CG step: fewer, heavier launches
    (2048, 512, 2048, 512, 512, 1),
    (1024, 512, 2048, 512, 512, 1),
    (1024, 1024, 2048, 512, 256, 1),
    (2048, 1024, 4096, 512, 512, 1),
    (4096, 512, 4096, 256, 512, 1),
    # one launch per CG step, LDS-staged, 6 vectors of traffic (2D batches;
    # others run the textbook form under these tiles)
    (4096, 512, 4096, 256, 256, 2),
    (4096, 512, 4096, 256, 512, 2),
    (2048, 512, 2048, 512, 512, 2),
    (2048, 1024, 4096, 512, 256, 2),
]

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sip_tiles.json")


def workload_key(field, shapes):
    ndim = max(len(s) for s in shapes)
    total = sum(math.prod(s) for s in shapes)
    return f"{field}|{ndim}d|n2^{int(round(math.log2(max(total, 1))))}|b2^{int(round(math.log2(len(shapes))))}"


def time_iterations(batch, iters):
    """Mean milliseconds per iteration of the batch (HIP graph replay, torch
    events on the current stream).  A first untimed run of the same length
    captures the graph."""
    import torch
    batch.run(iters)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    batch.run(iters)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / iters


def tune(batch, slots, ms, field, shapes, iters=8, candidates=CANDIDATES, cache=DEFAULT_CACHE, use_cache=True):
    """Pick tiles for `batch` (already holding the instances in `slots`, whose
    fields `ms` are used to reset the state between candidates).  Returns
    (best candidate, {candidate: ms per iteration})."""
    key = workload_key(field, shapes)
    if use_cache and cache and os.path.exists(cache):
        with open(cache) as f:
            known = json.load(f)
        if key in known:
            best = tuple(known[key]["tiles"])
            batch.set_tiles(*best)
            return best, known[key].get("timings", {})
    timings = {}
    for cand in candidates:
        batch.set_tiles(*cand)
        for sl, md in zip(slots, ms):
            batch.reset(sl, md)
        timings[cand] = time_iterations(batch, iters)
    best = min(timings, key=timings.get)
    batch.set_tiles(*best)
    for sl, md in zip(slots, ms):
        batch.reset(sl, md)
    if cache:
        known = {}
        if os.path.exists(cache):
            with open(cache) as f:
                known = json.load(f)
        known[key] = {"tiles": list(best), "timings": {",".join(map(str, c)): t for c, t in timings.items()}}
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        with open(cache, "w") as f:
            json.dump(known, f, indent=1)
    return best, {",".join(map(str, c)): t for c, t in timings.items()}
