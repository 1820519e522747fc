"""Edge cases of the boundary and the category thresholds (GPU), each through
the C ABI against the oracle:

- every threshold at its value and one either side: SORT rows are those with
  fewer than 1025 intermediate products; DENSE rows those whose column range
  fits the dense accumulator (2^13 columns for f64, 2^14 for f32); within a
  CHUNKED row, chunks of at least 1024 products take the dense accumulator
  and smaller ones are packed into sorts of at most 512 products (a chunk of
  513..1023 products is sorted alone) (Sections 3.1 and 3.4);
- 32-bit row pointers of C for a single product;
- MAGNUS_ERR_INDEX_OVERFLOW before any numeric launch;
- options.validate rejecting malformed CSR before anything indexes B;
- the one-call product magnus_spgemm and its memory;
- the plan's retry with narrower row batches when the allocator fails, and no
  leak when it keeps failing.
Integer-valued data makes every sum exact, so values compare bit for bit."""
import numpy as np
import pytest

import oracle
import workloads as wl
from workloads import CSR

from gpu_util import compare, gpu_product, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2501_07056_amd as mg
    c = mg.Context(0)
    yield c
    c.close()


def _one_entry_rows(col_lists, m, seed):
    """A has one row per list; row i has one entry per column of col_lists[i]
    (A_ij = integer in [-4, 4]) and B row j holds that single column with
    value 1, so row i's products land exactly on its listed columns."""
    rng = np.random.default_rng(seed)
    cols = np.concatenate([np.asarray(c, np.int64) for c in col_lists])
    n = len(cols)
    counts = [len(c) for c in col_lists]
    a = rng.integers(-4, 5, n).astype(np.float64)
    a[a == 0] = 1.0
    A = CSR(len(col_lists), n, np.concatenate([[0], np.cumsum(counts)]).astype(np.int64),
            np.arange(n, dtype=np.int32), a)
    B = CSR(n, m, np.arange(n + 1, dtype=np.int64), cols.astype(np.int32), np.ones(n))
    return A, B


def _rows_of_b(row_cols, m, seed, vt=np.float64):
    """A = identity-like (row i has one entry pointing at B row i, value in
    [-4, 4]); B row i holds the sorted distinct columns row_cols[i]."""
    rng = np.random.default_rng(seed)
    k = len(row_cols)
    a = rng.integers(1, 5, k).astype(vt)
    A = CSR(k, k, np.arange(k + 1, dtype=np.int64), np.arange(k, dtype=np.int32), a)
    lens = [len(c) for c in row_cols]
    colB = np.concatenate([np.sort(np.asarray(c, np.int64)) for c in row_cols]).astype(np.int32)
    valB = rng.integers(-4, 5, len(colB)).astype(vt)
    B = CSR(k, m, np.concatenate([[0], np.cumsum(lens)]).astype(np.int64), colB, valB)
    return A, B


def test_sort_threshold_1024_1025(ctx):
    """ip = 1024 is a SORT row, ip = 1025 is not (strict "fewer than"): with a
    narrow range it becomes DENSE, with a wide one CHUNKED."""
    rng = np.random.default_rng(101)
    narrow = lambda k: rng.choice(4096, k, replace=False)
    wide = lambda k: rng.choice(1 << 16, k, replace=False)
    A, B = _rows_of_b([narrow(1024), narrow(1025), wide(1025), wide(1024)], 1 << 16, 102)
    log("sort threshold 1024/1025")
    rp, col, val, info = gpu_product(ctx, A, B)
    assert info["rows_by_category"] == [2, 1, 1, 0]
    compare(rp, col, val, oracle.spgemm(A, B), np.float64, exact=True)


@pytest.mark.parametrize("vt,shift", [(np.float64, 13), (np.float32, 14)])
def test_dense_range_threshold(ctx, vt, shift):
    """A row whose column range is exactly the accumulator length (2^13 f64,
    2^14 f32) is DENSE; one column more makes it CHUNKED."""
    L = 1 << shift
    rng = np.random.default_rng(103)
    mid = rng.choice(np.arange(1, L - 1), 1500, replace=False)
    r0 = np.concatenate([[0, L - 1], mid])          # range L
    r1 = np.concatenate([[0, L], mid])              # range L + 1
    A, B = _rows_of_b([r0, r1], 4 * L, 104, vt)
    log(f"dense range threshold vt={vt.__name__}")
    rp, col, val, info = gpu_product(ctx, A, B)
    assert info["chunk_shift"] == shift
    assert info["rows_by_category"] == [0, 1, 1, 0]
    compare(rp, col, val, oracle.spgemm(A, B), vt, exact=True)


@pytest.mark.parametrize("shift", [13, 11])
def test_chunk_accumulator_thresholds(ctx, shift):
    """One CHUNKED row whose chunks hold 511, 1, 2, 512, 513, 1023, 1024,
    1025, 0 and 1 products (with repeated columns).  Chunks of >= 1024
    products take the dense accumulator (2 of them); the others are packed
    into sorts of at most 512 products: [511, 1], [2], [512], [513], [1023],
    [0, 1] (6 sort items)."""
    L = 1 << shift
    counts = [511, 1, 2, 512, 513, 1023, 1024, 1025, 0, 1]
    rng = np.random.default_rng(105)
    cols = []
    for c, k in enumerate(counts):
        cols.append(c * L + rng.integers(0, min(L, 700), k))
    A, B = _one_entry_rows([np.concatenate(cols), []], len(counts) * L, 106)
    log(f"chunk accumulator thresholds shift={shift}")
    rp, col, val, info = gpu_product(ctx, A, B, chunk_shift=shift)
    assert info["rows_by_category"] == [0, 0, 1, 1]
    assert info["n_bins"] == len(counts)
    assert info["n_dense_chunks"] == 2
    assert info["n_sort_groups"] == 6
    compare(rp, col, val, oracle.spgemm(A, B), np.float64, exact=True)
    ctx.set_options(chunk_shift=0)


@pytest.mark.parametrize("cat", ["auto", "sort", "dense", "chunked"])
def test_int32_c_rowptr_single_product(ctx, cat):
    """A single product written with 32-bit row pointers of C."""
    A, _ = wl.config2(11)
    Ai = CSR(A.nrows, A.ncols, A.rowptr, A.col, wl.values(A.nnz, wl.seed(107), "int", np.float64))
    log(f"int32 C rowptr cat={cat}")
    rp, col, val, info = gpu_product(ctx, Ai, Ai, rowptr_dtype="int32", force_category=cat)
    compare(rp, col, val, oracle.spgemm(Ai, Ai), np.float64, exact=True)
    ctx.set_options(force_category="auto")


def test_index_overflow_before_launch():
    """Config 3 at 2^24 rows: nnz(C) is about 2^32, so 32-bit row pointers of
    C cannot hold it.  magnus_execute returns MAGNUS_ERR_INDEX_OVERFLOW before
    it checks capacity or launches anything (C here has no room at all), and
    magnus_spgemm returns it without allocating C."""
    import torch

    import paper_2501_07056_amd as mg
    A, B = wl.config3(24)
    log("index overflow: config 3 at 2^24")
    dA, dB = mg.DeviceCSR.from_host(A), mg.DeviceCSR.from_host(B)
    del A, B
    ctx = mg.Context(0)
    try:
        p = ctx.plan(dA, dB)
        assert p.nnz > (1 << 31)
        dev = dA.rowptr.device
        C = mg.DeviceCSR(dA.nrows, dB.ncols, torch.zeros(dA.nrows + 1, dtype=torch.int32, device=dev),
                         torch.empty(0, dtype=torch.int32, device=dev),
                         torch.empty(0, dtype=torch.float32, device=dev))
        with pytest.raises(mg.MagnusError) as e:
            p.execute(C)
        assert e.value.name == "MAGNUS_ERR_INDEX_OVERFLOW"
        torch.cuda.synchronize()
        # nothing was written into C's row pointers
        assert int(C.rowptr.abs().sum()) == 0
        p.destroy()
        live = ctx.live_allocs
        with pytest.raises(mg.MagnusError) as e:
            ctx.spgemm_lib(dA, dB, rowptr_dtype=torch.int32)
        assert e.value.name == "MAGNUS_ERR_INDEX_OVERFLOW"
        assert ctx.live_allocs == live
    finally:
        ctx.close()


def test_validate_rejects_malformed_csr():
    """options.validate: a B row with columns out of order, a B column equal
    to ncols, an A column equal to A.ncols and a decreasing row pointer are
    each MAGNUS_ERR_INVALID_CSR; the check is read back before any pass
    indexes B by A's columns.  B's row-pointer buffer carries spare entries
    (equal to nnz) past its n + 1, so that even a read one past the end
    would stay inside it."""
    import torch

    import paper_2501_07056_amd as mg
    ctx = mg.Context(0, validate=1)
    dev = torch.device("cuda", 0)

    def dev_csr(nrows, ncols, rp, col, val, pad=0):
        rp = np.asarray(rp, np.int64)
        rpt = torch.from_numpy(np.concatenate([rp, np.full(pad, rp[-1])])).to(dev)
        return mg.DeviceCSR(nrows, ncols, rpt, torch.from_numpy(np.asarray(col, np.int32)).to(dev),
                            torch.from_numpy(np.asarray(val, np.float64)).to(dev))

    try:
        A = dev_csr(3, 4, [0, 2, 3, 4], [0, 2, 1, 3], [1, 2, 3, 4])
        B = dev_csr(4, 6, [0, 2, 3, 5, 6], [1, 4, 0, 2, 5, 3], [1, 1, 1, 1, 1, 1], pad=8)
        p = ctx.plan(A, B)  # well formed: accepted
        C = p.execute()
        torch.cuda.synchronize()
        p.destroy()
        Ah = CSR(3, 4, np.array([0, 2, 3, 4]), np.array([0, 2, 1, 3], np.int32), np.array([1., 2, 3, 4]))
        Bh = CSR(4, 6, np.array([0, 2, 3, 5, 6]), np.array([1, 4, 0, 2, 5, 3], np.int32), np.ones(6))
        rp, col, val = C.to_host()
        compare(rp.astype(np.int64), col.astype(np.int64), val, oracle.spgemm(Ah, Bh), np.float64,
                exact=True)
        bad = {
            "B row out of order": (A, dev_csr(4, 6, [0, 2, 3, 5, 6], [4, 1, 0, 2, 5, 3], [1] * 6, 8)),
            "B column == ncols": (A, dev_csr(4, 6, [0, 2, 3, 5, 6], [1, 6, 0, 2, 5, 3], [1] * 6, 8)),
            "A column == ncols": (dev_csr(3, 4, [0, 2, 3, 4], [0, 2, 1, 4], [1, 2, 3, 4]), B),
            "A rowptr decreasing": (dev_csr(3, 4, [0, 3, 2, 4], [0, 2, 1, 3], [1, 2, 3, 4]), B),
        }
        for what, (a, b) in bad.items():
            log(f"validate: {what}")
            with pytest.raises(mg.MagnusError) as e:
                ctx.plan(a, b)
            assert e.value.name == "MAGNUS_ERR_INVALID_CSR", what
        assert ctx.live_allocs == 0
    finally:
        ctx.close()


@pytest.mark.parametrize("rpt", ["int64", "int32"])
def test_spgemm_one_call(rpt):
    """magnus_spgemm allocates C through the registered allocator (torch's
    caching allocator here) and magnus_csr_free returns it."""
    import torch

    import paper_2501_07056_amd as mg
    A, _ = wl.config2(12)
    log(f"magnus_spgemm rowptr={rpt}")
    ctx = mg.Context(0)
    try:
        dA = mg.DeviceCSR.from_host(A)
        C = ctx.spgemm_lib(dA, dA, rowptr_dtype=getattr(torch, rpt))
        assert ctx.live_allocs == 3
        D = C.to_device_csr()
        torch.cuda.synchronize()
        rp, col, val = D.to_host()
        compare(rp.astype(np.int64), col.astype(np.int64), val.astype(np.float64),
                oracle.spgemm(A, A), np.float64, exact=False)
        C.free()
        assert ctx.live_allocs == 0
    finally:
        ctx.close()


def test_oom_retry_and_no_leak():
    """An allocator that refuses the full-width workspace makes the plan retry
    with row batches half as wide, which succeeds (more batches, same C).  An
    allocator that fails after k allocations ends in MAGNUS_ERR_OOM with every
    allocation it made returned."""
    import paper_2501_07056_amd as mg
    A, _ = wl.config2(12)
    ipt = int(oracle.ip(A, A).sum())
    ref = oracle.spgemm(A, A)
    # the workspace of one batch of all products holds 8 bytes of value each
    limit = 6 * ipt
    log(f"oom retry: ip={ipt}, allocations >= {limit} bytes refused")
    ctx = mg.Context(0, alloc_filter=lambda n: n < limit)
    try:
        rp, col, val, info = gpu_product(ctx, A, A, force_category="chunked", batch_products=ipt,
                                         chunk_runs=-1)
        assert info["n_batches"] >= 2
        compare(rp, col, val, ref, np.float64, exact=False)
        assert ctx.live_allocs == 0
    finally:
        ctx.close()
    for k in (0, 1, 3, 8, 20):
        state = {"left": k}

        def filt(n):
            state["left"] -= 1
            return state["left"] >= 0

        ctx = mg.Context(0, alloc_filter=filt)
        try:
            log(f"oom after {k} allocations")
            with pytest.raises(mg.MagnusError) as e:
                gpu_product(ctx, A, A, force_category="chunked", batch_products=ipt,
                            chunk_runs=(-1 if k % 2 else 1))
            assert e.value.name == "MAGNUS_ERR_OOM"
            assert ctx.live_allocs == 0
        finally:
            ctx.close()
