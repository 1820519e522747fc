"""Deterministic mode (GPU): with the `deterministic` option every value of C
must equal, bit for bit, the oracle's input-precision sum, which adds the
products of Eq. 1 in stored order (each entry of A's row in order, each entry
of the B row in order, from +0.0).  Random values, so any other summation
order would show up as differing low bits."""
import numpy as np
import pytest

import oracle
import workloads as wl
from workloads import CSR

from gpu_util import compare, gpu_product, log

pytestmark = pytest.mark.gpu


@pytest.fixture()
def ctx():
    import paper_2501_07056_amd as mg
    c = mg.Context(0, deterministic=1)
    yield c
    c.close()


def test_det_rmat_default(ctx):
    A, _ = wl.config2(11)
    log("det rmat11 defaults")
    rp, col, val, info = gpu_product(ctx, A, A)
    ref = oracle.spgemm(A, A)
    compare(rp, col, val, ref, np.float64, exact=True)
    # every non-empty row went through the CHUNKED path
    assert info["rows_by_category"][0] == 0 and info["rows_by_category"][1] == 0
    assert info["coarse_rows"] == 0


def test_det_rmat_many_chunks_tiles_batches(ctx):
    """Rows spanning many chunks and many tiles, several batches, dense and
    packed-sort chunks mixed."""
    A, _ = wl.config2(12)
    log("det rmat12 shift=6 tile=512 dense_min=64")
    rp, col, val, info = gpu_product(ctx, A, A, chunk_shift=6, tile_products=512,
                                     bin_dense_min=64, batch_products=200000)
    assert info["n_batches"] > 1
    compare(rp, col, val, oracle.spgemm(A, A), np.float64, exact=True)
    # the same bits again
    rp2, col2, val2, _ = gpu_product(ctx, A, A)
    assert np.array_equal(rp, rp2) and np.array_equal(col, col2)
    assert np.array_equal(val.view(np.int64), val2.view(np.int64))


@pytest.mark.parametrize("vt", [np.float64, np.float32])
def test_det_er(ctx, vt):
    A = wl.erdos_renyi(3000, 5000, 12, wl.seed(80), val_dtype=vt)
    B = wl.erdos_renyi(5000, 20000, 20, wl.seed(81), val_dtype=vt)
    log(f"det er vt={vt.__name__}")
    rp, col, val, info = gpu_product(ctx, A, B, chunk_shift=10)
    compare(rp, col, val, oracle.spgemm(A, B), vt, exact=True)


def test_det_long_runs_dense(ctx):
    """Few columns, many products each: long runs of equal columns inside
    every 64-product window of the ordered dense accumulator."""
    A = wl.erdos_renyi(400, 300, 64, wl.seed(82))
    B = wl.erdos_renyi(300, 16, 8, wl.seed(83))
    log("det long runs")
    rp, col, val, info = gpu_product(ctx, A, B, bin_dense_min=32)
    compare(rp, col, val, oracle.spgemm(A, B), np.float64, exact=True)


def test_det_table_symbolic_and_wide_types(ctx):
    """Symbolic phase without the row bitmap (small LDS budget), 64-bit row
    pointers and columns, f32 values."""
    A = wl.erdos_renyi(2000, 6000, 10, wl.seed(84), val_dtype=np.float32,
                       rowptr_dtype=np.int64, col_dtype=np.int64)
    B = wl.erdos_renyi(6000, 9000, 14, wl.seed(85), val_dtype=np.float32,
                       rowptr_dtype=np.int64, col_dtype=np.int64)
    log("det table symbolic, int64 indices, f32")
    rp, col, val, info = gpu_product(ctx, A, B, chunk_shift=8, lds_bytes=16384)
    compare(rp, col, val, oracle.spgemm(A, B), np.float32, exact=True)


def test_det_edge_cases(ctx):
    """Empty product, 1x1, cancellation to +0.0, -0.0 products, and empty
    rows of A and of B in a 50000-column product of 256-column chunks."""
    log("det edge cases")
    E = CSR(0, 5, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    B = wl.erdos_renyi(5, 7, 2, wl.seed(85))
    rp, col, val, info = gpu_product(ctx, E, B)
    assert len(rp) == 1 and rp[0] == 0 and len(col) == 0
    one = CSR(1, 1, np.array([0, 1]), np.array([0], np.int32), np.array([3.0]))
    rp, col, val, info = gpu_product(ctx, one, one)
    assert list(rp) == [0, 1] and list(col) == [0] and list(val) == [9.0]
    A = CSR(2, 2, np.array([0, 2, 3]), np.array([0, 1, 0], np.int32), np.array([1.0, 1.0, 1.0]))
    Bm = CSR(2, 1, np.array([0, 1, 2]), np.array([0, 0], np.int32), np.array([2.0, -2.0]))
    rp, col, val, info = gpu_product(ctx, A, Bm)
    assert list(col) == [0, 0] and val[0] == 0.0 and not np.signbit(val[0]) and val[1] == 2.0
    Bz = CSR(2, 1, np.array([0, 1, 2]), np.array([0, 0], np.int32), np.array([-0.0, -0.0]))
    rp, col, val, info = gpu_product(ctx, A, Bz)
    assert not np.signbit(val).any()
    A = wl.erdos_renyi(400, 300, 5, wl.seed(86))
    rpA = A.rowptr.astype(np.int64).copy()
    keep = np.ones(A.nnz, bool)
    for i in range(0, 400, 7):
        keep[rpA[i]:rpA[i + 1]] = False
    cnt = np.array([keep[rpA[i]:rpA[i + 1]].sum() for i in range(400)])
    A2 = CSR(400, 300, np.concatenate([[0], np.cumsum(cnt)]), A.col[keep], A.val[keep])
    Bs = wl.erdos_renyi(300, 50000, 7, wl.seed(87))
    rpB = Bs.rowptr.astype(np.int64)
    keepB = np.ones(Bs.nnz, bool)
    for j in range(0, 300, 5):
        keepB[rpB[j]:rpB[j + 1]] = False
    cntB = np.array([keepB[rpB[j]:rpB[j + 1]].sum() for j in range(300)])
    B2 = CSR(300, 50000, np.concatenate([[0], np.cumsum(cntB)]), Bs.col[keepB], Bs.val[keepB])
    rp, col, val, info = gpu_product(ctx, A2, B2, chunk_shift=8)
    compare(rp, col, val, oracle.spgemm(A2, B2), np.float64, exact=True)


def test_det_rejected_by_batch_plans(ctx):
    import paper_2501_07056_amd as mg
    A = wl.erdos_renyi(100, 100, 4, wl.seed(86))
    dA = mg.DeviceCSR.from_host(A)
    with pytest.raises(Exception):
        ctx.batch_plan([(dA, dA)])
