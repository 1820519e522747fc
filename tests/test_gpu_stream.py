"""The chunk building blocks on one stream of products (the microbenchmark
entry point, Section 4.1), against the oracle: a stream (c_j, v_j) is the
intermediate product of the 1 x n row (v_j) times the n x m matrix whose row
j holds the single entry (c_j, 1), so its per-column sums are that product's
row.  Structure exactly; values bit-exact on integers, else within rtol *
sum|v|."""
import numpy as np
import pytest

import oracle
from workloads import CSR

from gpu_util import RTOL, log

pytestmark = pytest.mark.gpu


def _stream(n, m, seed, vt, integer=False, hot=0):
    rng = np.random.default_rng(seed)
    cols = rng.integers(0, m, size=n)
    if hot:  # a few heavy columns, as in a power-law row
        cols[: n // 4] = rng.integers(0, hot, size=n // 4)
        rng.shuffle(cols)
    vals = (rng.integers(-4, 5, size=n) if integer else rng.uniform(-1, 1, size=n)).astype(vt)
    return cols.astype(np.int32), vals


def _reference(cols, vals, m):
    n = len(cols)
    A = CSR(1, n, np.array([0, n], np.int64), np.arange(n, dtype=np.int32), vals)
    B = CSR(n, m, np.arange(n + 1, dtype=np.int64), cols.astype(np.int32),
            np.ones(n, dtype=vals.dtype))
    return oracle.spgemm(A, B)


@pytest.fixture(scope="module")
def ctx():
    import paper_2501_07056_amd as mg
    c = mg.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("vt", [np.float64, np.float32])
@pytest.mark.parametrize("dense_min", [0, 1, 1025])
def test_stream_matches_oracle(ctx, vt, dense_min):
    import torch
    shift = 12 if vt == np.float64 else 13
    for n, m, hot in ((300_000, 1 << 20, 0), (200_000, (1 << 19) + 77, 3000), (5, 1000, 0)):
        cols, vals = _stream(n, m, n + m, vt, hot=hot)
        log(f"stream n={n} m={m} vt={vt.__name__} dense_min={dense_min}")
        oc, ov, t = ctx.stream_chunks(torch.from_numpy(cols).cuda(), torch.from_numpy(vals).cuda(),
                                      m, shift, dense_min)
        ref = _reference(cols, vals, m)
        gc, gv = oc.cpu().numpy().astype(np.int64), ov.cpu().numpy().astype(np.float64)
        assert np.array_equal(gc, ref.col)
        assert not np.signbit(gv[gv == 0]).any()
        assert (np.abs(gv - ref.ref) <= RTOL[np.dtype(vt)] * ref.abssum).all()
        assert t["chunks"] == ((m - 1) >> shift) + 1
        if dense_min == 1:
            assert t["sort_groups"] == 0
        if dense_min == 1025 and n < 1024 * t["chunks"]:
            assert t["sort_groups"] > 0


def test_stream_integers_exact_and_errors(ctx):
    import torch

    import paper_2501_07056_amd as mg
    cols, vals = _stream(1 << 20, 1 << 18, 7, np.float64, integer=True, hot=100)
    oc, ov, t = ctx.stream_chunks(torch.from_numpy(cols).cuda(), torch.from_numpy(vals).cuda(),
                                  1 << 18, 12)
    ref = _reference(cols, vals, 1 << 18)
    assert np.array_equal(oc.cpu().numpy().astype(np.int64), ref.col)
    assert np.array_equal(ov.cpu().numpy(), ref.val)
    assert min(t["histogram_ms"], t["reorder_ms"], t["accumulate_ms"]) > 0
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    oc, ov, t = ctx.stream_chunks(e, torch.empty(0, dtype=torch.float64, device="cuda"), 10, 4)
    assert oc.numel() == 0
    c1 = torch.zeros(4, dtype=torch.int32, device="cuda")
    v1 = torch.ones(4, dtype=torch.float64, device="cuda")
    with pytest.raises(mg.MagnusError):  # 2^20 chunks of 2^4 columns
        ctx.stream_chunks(c1, v1, 1 << 24, 4)
    with pytest.raises(mg.MagnusError):  # accumulator of 2^16 doubles exceeds the LDS
        ctx.stream_chunks(c1, v1, 1 << 20, 16)
