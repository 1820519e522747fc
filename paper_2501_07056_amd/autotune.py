"""Autotuner for batches of products.

The choices of the method that depend on the input are tuned by timing them
on the device:

* the SORT threshold of each product (rows with fewer intermediate products
  than the threshold are sorted, the others use a dense accumulator or the
  chunk reorder; Section 3.1 derives it from cache sizes, here it is
  searched), per size class of product, among the thresholds that keep the
  class's rows out of the CHUNKED category when there are such (a product
  with CHUNKED rows is planned on its own, outside the batch's launches);
* the threads per row block: the workgroup size of the dense accumulators,
  for the whole batch;
* when the batch has CHUNKED rows (Algorithm 3): the chunk length, i.e. the
  chunk count per row (Section 3.5), the per-chunk threshold between the
  dense accumulator and the sort (Section 3.4), and the products per packed
  sort of small chunks, for the whole batch, one after the other
  (coordinate descent from the library's defaults).

A size class is (value type, log2 of the row count, log2 of the mean row
length of A and of B), all rounded.  For each class, up to `per_class`
products of the batch are planned and executed as a sub-batch under every
candidate threshold; the fastest median of `reps` timed runs (plan plus
execute, events on the stream) wins.  Results are cached in a JSON file keyed
by the device's gfx architecture and class, so a later batch of the same
classes reuses them without timing anything.
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
# CHUNKED rows: chunk length relative to the gfx950 default (2^13 columns for
# f64, 2^14 for f32), per-chunk dense threshold, products per packed sort
CHUNK_SHIFT_DELTAS = (0, -1, -2)
BIN_DENSE_MIN_CANDIDATES = (256, 512, 1024)
SORT_GROUP_CANDIDATES = (256, 512, 1024)


def device_arch(device) -> str:
    """The gfx architecture of `device` (e.g. gfx950), the tuning cache key."""
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", "") or ""
    return arch.split(":")[0] or torch.cuda.get_device_name(device)


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


def _time_batch(ctx, pairs, sort_max, reps, stream, info=None):
    """Median device milliseconds of plan + execute of `pairs` as one batch
    (the first run's plan info is stored in info when given)."""
    ts = []
    for r in range(reps + 1):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record(stream)
            bp = ctx.batch_plan(pairs, sort_max=sort_max, stream=stream)
            try:
                if info is not None and r == 0:
                    info.update(bp.info.as_dict())
                bp.execute(stream=stream)
            finally:
                e1.record(stream)
                stream.synchronize()
                bp.destroy()
        if r > 0:  # the first run captures the graph and warms the allocator
            ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def _default_shift(pairs) -> int:
    import paper_2501_07056_amd as mg
    f64 = str(pairs[0][0].val.dtype).endswith("float64")
    lds = torch.cuda.get_device_properties(pairs[0][0].rowptr.device).shared_memory_per_block
    return mg.gpu_chunk_shift(f64, lds)


def tune(ctx, pairs, cache_path=None, per_class=8, reps=3, candidates=SORT_MAX_CANDIDATES,
         blocks=DENSE_BLOCK_CANDIDATES, log=None):
    """Pick per-product SORT thresholds and the dense workgroup size for the
    batch `pairs` (list of (A, B) DeviceCSR).  Returns
    {"sort_max": [per product], "dense_block": int, "classes": {...}}."""
    dev = device_arch(pairs[0][0].rowptr.device) if pairs else "none"
    cache = _load(cache_path)
    entry = cache.setdefault(dev, {"classes": {}, "dense_block": {}})
    entry.setdefault("chunked", {})
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
        times, chunked = {}, {}
        for sm in candidates:
            info = {}
            times[str(sm)] = _time_batch(ctx, sub, [sm] * len(sub), reps, stream, info)
            chunked[str(sm)] = info.get("rows_by_category", [0, 0, 0, 0])[2]
        # a product with CHUNKED rows is planned on its own and leaves the
        # batch's shared launches: thresholds that keep the class's rows SORT
        # or DENSE win when there are any
        keep = [k for k in times if chunked[k] == 0] or list(times)
        best = min(keep, key=times.get)
        entry["classes"][key] = {"sort_max": int(best), "ms": times, "products": len(sub),
                                 "chunked_rows": chunked}
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
    dense_block = entry["dense_block"][bkey]["dense_block"]
    # CHUNKED rows: chunk length, per-chunk dense threshold, packed sort size
    if bkey not in entry["chunked"]:
        step = max(1, len(pairs) // (4 * per_class))
        sel = list(range(0, len(pairs), step))
        sample = [pairs[i] for i in sel]
        sm_sample = [sort_max[i] for i in sel]
        saved_opts = {k: getattr(ctx.opts, k) for k in
                      ("dense_block", "chunk_shift", "bin_dense_min", "sort_group_max")}
        choice = {"chunk_shift": 0, "bin_dense_min": 0, "sort_group_max": 0}
        rec = {"searched": False}
        try:
            ctx.set_options(dense_block=dense_block)
            info = {}
            base = _time_batch(ctx, sample, sm_sample, reps, stream, info)
            if info.get("rows_by_category", [0, 0, 0, 0])[2] > 0:
                rec["searched"] = True
                d0 = _default_shift(pairs)
                grid = (("chunk_shift", [d0 + d for d in CHUNK_SHIFT_DELTAS if d0 + d >= 6]),
                        ("bin_dense_min", list(BIN_DENSE_MIN_CANDIDATES)),
                        ("sort_group_max", list(SORT_GROUP_CANDIDATES)))
                best = base
                for name, cands in grid:
                    times = {}
                    for v in cands:
                        ctx.set_options(**{**choice, name: v})
                        times[str(v)] = _time_batch(ctx, sample, sm_sample, reps, stream)
                    v = min(times, key=times.get)
                    if times[v] < best:
                        best = times[v]
                        choice[name] = int(v)
                    rec[name] = times
                    if log:
                        log(f"autotune {name}: {times}")
        finally:
            ctx.set_options(**saved_opts)
        rec.update(choice)
        entry["chunked"][bkey] = rec
    ch = entry["chunked"][bkey]
    _save(cache_path, cache)
    if log:
        log(f"autotune done in {time.time() - t0:.1f}s")
    return {"sort_max": sort_max, "dense_block": dense_block,
            "chunk_shift": ch["chunk_shift"], "bin_dense_min": ch["bin_dense_min"],
            "sort_group_max": ch["sort_group_max"], "arch": dev,
            "classes": {k: entry["classes"][k] for k in classes}}
