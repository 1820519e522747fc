"""The batch autotuner (GPU): it picks thresholds from its candidate set,
caches them per size class, answers a second call from the cache without
timing anything, and the batch planned with its choices matches the oracle."""
import numpy as np
import pytest

import oracle
import workloads as wl

from gpu_util import compare, log

pytestmark = pytest.mark.gpu


def test_autotune_cache_and_parity(tmp_path, monkeypatch):
    import torch

    import paper_2501_07056_amd as mg
    from paper_2501_07056_amd import autotune
    ctx = mg.Context(0)
    try:
        pairs_host = []
        for b, (n, d) in enumerate(wl.config4_shapes(10, 128, 4096, 4, 32)):
            A = wl.erdos_renyi(n, n, d, wl.seed(2000 + b), val_dtype=np.float32,
                               rowptr_dtype=np.int32, col_dtype=np.int32)
            pairs_host.append((A, A))
        pairs = []
        for A, _ in pairs_host:
            dA = mg.DeviceCSR.from_host(A)
            pairs.append((dA, dA))
        cache = str(tmp_path / "tune.json")
        log("autotune first call")
        t = autotune.tune(ctx, pairs, cache_path=cache, per_class=2, reps=1)
        assert len(t["sort_max"]) == len(pairs)
        assert set(t["sort_max"]) <= set(autotune.SORT_MAX_CANDIDATES)
        assert t["dense_block"] in autotune.DENSE_BLOCK_CANDIDATES
        assert ctx.opts.dense_block == 0  # restored
        assert t["arch"].startswith("gfx")
        # ER rows of this batch are SORT or DENSE under every threshold tried
        # here only if no row is CHUNKED; either way the knobs are valid
        assert t["chunk_shift"] == 0 or 6 <= t["chunk_shift"] <= 16
        assert t["bin_dense_min"] in (0,) + autotune.BIN_DENSE_MIN_CANDIDATES
        assert t["sort_group_max"] in (0,) + autotune.SORT_GROUP_CANDIDATES

        def no_timing(*a, **k):
            raise AssertionError("cached classes must not be timed again")
        monkeypatch.setattr(autotune, "_time_batch", no_timing)
        t2 = autotune.tune(ctx, pairs, cache_path=cache, per_class=2, reps=1)
        assert t2["sort_max"] == t["sort_max"] and t2["dense_block"] == t["dense_block"]

        ctx.set_options(dense_block=t["dense_block"], chunk_shift=t["chunk_shift"],
                        bin_dense_min=t["bin_dense_min"], sort_group_max=t["sort_group_max"])
        bp = ctx.batch_plan(pairs, sort_max=t["sort_max"])
        try:
            outs = bp.execute()
            torch.cuda.synchronize()
            for C, (A, B) in zip(outs, pairs_host):
                rp, col, val = C.to_host()
                compare(rp.astype(np.int64), col.astype(np.int64), val.astype(np.float64),
                        oracle.spgemm(A, B), np.float32, exact=False)
        finally:
            bp.destroy()
    finally:
        ctx.close()


def test_autotune_chunked_batch(tmp_path):
    """A batch with CHUNKED rows (wide R-MAT and ER products): the chunk
    length, the per-chunk dense threshold and the packed sort size are
    searched, cached under the gfx architecture, and the batch planned with
    the choices matches the oracle."""
    import json

    import torch

    import paper_2501_07056_amd as mg
    from paper_2501_07056_amd import autotune
    ctx = mg.Context(0)
    try:
        R, _ = wl.config2(12)
        er = dict(rowptr_dtype=np.int32, col_dtype=np.int32, val_dtype=np.float64)
        # ER rows of 40 x 40 = 1600 products over 2^16 columns are CHUNKED
        # under every SORT threshold tried
        pairs_host = [(R, R)] + [(wl.erdos_renyi(400, 400, 40, wl.seed(2100 + b), **er),
                                  wl.erdos_renyi(400, 1 << 16, 40, wl.seed(2200 + b), **er))
                                 for b in range(3)]
        pairs = [(mg.DeviceCSR.from_host(A), mg.DeviceCSR.from_host(B)) for A, B in pairs_host]
        cache = str(tmp_path / "tune.json")
        log("autotune chunked batch")
        t = autotune.tune(ctx, pairs, cache_path=cache, per_class=2, reps=1,
                          candidates=(1025, 65))
        data = json.load(open(cache))
        assert list(data) == [t["arch"]] and t["arch"].startswith("gfx")
        rec = list(data[t["arch"]]["chunked"].values())[0]
        assert rec["searched"] and "chunk_shift" in rec and "bin_dense_min" in rec
        ctx.set_options(dense_block=t["dense_block"], chunk_shift=t["chunk_shift"],
                        bin_dense_min=t["bin_dense_min"], sort_group_max=t["sort_group_max"])
        bp = ctx.batch_plan(pairs, sort_max=t["sort_max"])
        try:
            outs = bp.execute()
            torch.cuda.synchronize()
            for C, (A, B) in zip(outs, pairs_host):
                rp, col, val = C.to_host()
                compare(rp.astype(np.int64), col.astype(np.int64), val.astype(np.float64),
                        oracle.spgemm(A, B), np.float64, exact=False)
        finally:
            bp.destroy()
    finally:
        ctx.close()
