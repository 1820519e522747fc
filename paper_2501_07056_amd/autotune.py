"""Autotuner for batches of products.

Two choices of the method are tuned by timing them on the device:

* the SORT/DENSE threshold of each product (rows with fewer intermediate
  products than the threshold are sorted, the others use the dense
  accumulator; Section 3.1 sets it from the cache-line count of the row's
  dense accumulator, here it is searched), per size class of product;
* the workgroup size of the dense accumulator, for the whole batch.

A size class is (value type, log2 of the row count, log2 of the mean row
length of A and of B), all rounded.  For each class, up to `per_class`
products of the batch are planned and executed as a sub-batch under every
candidate threshold; the fastest median of `reps` timed runs (plan plus
execute, events on the stream) wins.  Results are cached in a JSON file keyed
by device name and class, so a later batch of the same classes reuses them
without timing anything.
"""
from __future__ import annotations

import json
import math
import os
import time
import zlib

import torch

SORT_MAX_CANDIDATES = (1, 65, 257, 1025)
DENSE_BLOCK_CANDIDATES = (256, 512, 1024)


def size_class(A, B) -> str:
    """Class key of the product A*B (DeviceCSR or host CSR)."""
    vt = "f64" if str(getattr(A.val, "dtype", "")).endswith("float64") else "f32"
    n = max(int(A.nrows), 1)
    da = max(int(A.nnz), 1) / n
    db = max(int(B.nnz), 1) / max(int(B.nrows), 1)
    return f"{vt}/n{round(math.log2(n))}/da{round(math.log2(da))}/db{round(math.log2(db))}"


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _save(path, data):
    if not path:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_batch(ctx, pairs, sort_max, reps, stream):
    """Median device milliseconds of plan + execute of `pairs` as one batch."""
    ts = []
    for r in range(reps + 1):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record(stream)
            bp = ctx.batch_plan(pairs, sort_max=sort_max, stream=stream)
            try:
                bp.execute(stream=stream)
            finally:
                e1.record(stream)
                stream.synchronize()
                bp.destroy()
        if r > 0:  # the first run captures the graph and warms the allocator
            ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def tune(ctx, pairs, cache_path=None, per_class=8, reps=3, candidates=SORT_MAX_CANDIDATES,
         blocks=DENSE_BLOCK_CANDIDATES, log=None):
    """Pick per-product SORT thresholds and the dense workgroup size for the
    batch `pairs` (list of (A, B) DeviceCSR).  Returns
    {"sort_max": [per product], "dense_block": int, "classes": {...}}."""
    dev = torch.cuda.get_device_name(pairs[0][0].rowptr.device) if pairs else "none"
    cache = _load(cache_path)
    entry = cache.setdefault(dev, {"classes": {}, "dense_block": {}})
    classes = {}
    for i, (A, B) in enumerate(pairs):
        classes.setdefault(size_class(A, B), []).append(i)
    stream = torch.cuda.Stream(device=pairs[0][0].rowptr.device) if pairs else None
    saved = ctx.opts.dense_block
    t0 = time.time()
    for key, idx in sorted(classes.items()):
        if key in entry["classes"]:
            continue
        sub = [pairs[i] for i in idx[:per_class]]
        times = {}
        for sm in candidates:
            times[str(sm)] = _time_batch(ctx, sub, [sm] * len(sub), reps, stream)
        best = min(times, key=times.get)
        entry["classes"][key] = {"sort_max": int(best), "ms": times, "products": len(sub)}
        if log:
            log(f"autotune {key}: sort_max={best} ({times})")
    sort_max = [entry["classes"][size_class(A, B)]["sort_max"] for A, B in pairs]
    # the dense workgroup size is one option for the whole batch
    bkey = ",".join(f"{k}x{len(v)}" for k, v in sorted(classes.items()))
    bkey = f"{len(pairs)}:{zlib.crc32(bkey.encode()):08x}"
    if bkey not in entry["dense_block"]:
        step = max(1, len(pairs) // (4 * per_class))
        sel = list(range(0, len(pairs), step))
        sample = [pairs[i] for i in sel]
        sm_sample = [sort_max[i] for i in sel]
        times = {}
        try:
            for b in blocks:
                ctx.set_options(dense_block=b)
                times[str(b)] = _time_batch(ctx, sample, sm_sample, reps, stream)
        finally:
            ctx.set_options(dense_block=saved)
        entry["dense_block"][bkey] = {"dense_block": int(min(times, key=times.get)), "ms": times}
        if log:
            log(f"autotune dense_block: {entry['dense_block'][bkey]}")
    _save(cache_path, cache)
    if log:
        log(f"autotune done in {time.time() - t0:.1f}s")
    return {"sort_max": sort_max, "dense_block": entry["dense_block"][bkey]["dense_block"],
            "classes": {k: entry["classes"][k] for k in classes}}
