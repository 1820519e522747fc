"""Parity of the HIP path with the CPU oracle (GPU).  Every case runs the
product through the C ABI and compares element by element: structure exactly,
values bit-exactly on integer data and within rtol * sum|a_ik b_kj| otherwise
(rtol 1e-12 for f64, 1e-5 for f32)."""
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


CATS = ["auto", "sort", "dense", "chunked"]


@pytest.mark.parametrize("cat", CATS)
def test_config1_bit_exact(ctx, cat):
    A, B = wl.config1()
    log(f"config1 cat={cat}")
    rp, col, val, info = gpu_product(ctx, A, B, force_category=cat)
    ref = oracle.spgemm(A, B)
    compare(rp, col, val, ref, np.float64, exact=True)
    assert info["ip_total"] == 262144
    assert info["nnz_c"] == ref.nnz


@pytest.mark.parametrize("cat", CATS)
@pytest.mark.parametrize("vt", [np.float64, np.float32])
def test_er_random_values(ctx, cat, vt):
    A = wl.erdos_renyi(3000, 5000, 12, wl.seed(80), val_dtype=vt)
    B = wl.erdos_renyi(5000, 20000, 20, wl.seed(81), val_dtype=vt)
    log(f"er cat={cat} vt={vt.__name__}")
    rp, col, val, info = gpu_product(ctx, A, B, force_category=cat)
    compare(rp, col, val, oracle.spgemm(A, B), vt, exact=False)


@pytest.mark.parametrize("cat", CATS)
def test_rmat_mixed(ctx, cat):
    A, _ = wl.config2(11)
    log(f"rmat11 cat={cat}")
    rp, col, val, info = gpu_product(ctx, A, A, force_category=cat)
    compare(rp, col, val, oracle.spgemm(A, A), np.float64, exact=False)


def test_rmat_auto_small_chunks(ctx):
    """Small chunk length so CHUNKED rows span many chunks and tiles."""
    A, _ = wl.config2(12)
    log("rmat12 shift=8 tile=512")
    rp, col, val, info = gpu_product(ctx, A, A, force_category="chunked", chunk_shift=8,
                                     tile_products=512, batch_products=200000, chunk_runs=-1)
    assert info["n_batches"] > 1 and info["run_binned"] == 0
    compare(rp, col, val, oracle.spgemm(A, A), np.float64, exact=False)
    ctx.set_options(chunk_shift=0, tile_products=0, batch_products=0, chunk_runs=0)


def test_rmat_table_symbolic(ctx):
    """LDS budget too small for a whole row's bitmap: the symbolic phase of
    CHUNKED rows goes through per-tile histograms, reorder and per-chunk
    counting instead."""
    A, _ = wl.config2(12)
    log("rmat12 table symbolic")
    for shift in (8, 10):
        rp, col, val, info = gpu_product(ctx, A, A, force_category="chunked", chunk_shift=shift,
                                         tile_products=1024, lds_bytes=16384,
                                         batch_products=300000, chunk_runs=-1)
        assert info["run_binned"] == 0
        compare(rp, col, val, oracle.spgemm(A, A), np.float64, exact=False)
    ctx.set_options(chunk_shift=0, tile_products=0, batch_products=0, lds_bytes=0,
                    force_category="auto", chunk_runs=0)


@pytest.mark.parametrize("vt", [np.float64, np.float32])
def test_coarse_level_er(ctx, vt):
    """Rows wider than one coarse chunk take the coarse level (Section 3.3):
    small coarse chunks (4 chunks of 2^9 columns under a 16 KiB LDS budget)
    put every CHUNKED row through both reorders; the ablation without the
    coarse level gives the same product."""
    A = wl.erdos_renyi(3000, 5000, 12, wl.seed(88), val_dtype=vt)
    B = wl.erdos_renyi(5000, 1 << 18, 100, wl.seed(89), val_dtype=vt)
    ref = oracle.spgemm(A, B)
    log(f"coarse er vt={vt.__name__}")
    # 4 / 64 chunks per coarse chunk with the first workspace kept between
    # the phases; 64 under a 2 MiB workspace cap (first reorder redone in the
    # numeric phase, many batches); the coarse level off
    for cc, cap in ((4, 0), (64, 0), (64, 2 << 20), (-1, 0)):
        rp, col, val, info = gpu_product(ctx, A, B, force_category="chunked", lds_bytes=16384,
                                         coarse_chunks=cc, batch_products=0 if cap else 400000,
                                         max_workspace_bytes=cap)
        if cc > 0:
            assert info["coarse_rows"] == A.nrows and info["coarse_chunks"] > A.nrows
            assert info["rows_by_category"][2] == A.nrows and info["n_batches"] == 0
            # every coarse chunk holds at most 1024 products: all are sorted
            # directly, none goes through the fine level
            assert info["coarse_fine_chunks"] == 0
        else:
            assert info["coarse_rows"] == 0
        compare(rp, col, val, ref, vt, exact=False)
    ctx.set_options(force_category="auto", lds_bytes=0, coarse_chunks=0, batch_products=0,
                    max_workspace_bytes=0)


def test_coarse_level_rmat(ctx):
    """Power-law rows through the coarse level: chunks of 2^6 columns, coarse
    chunks of 4 of them, so heavy rows span many coarse chunks (some empty)
    and some fine chunks are dense; several batches."""
    A, _ = wl.config2(12)
    log("coarse rmat12")
    rp, col, val, info = gpu_product(ctx, A, A, force_category="chunked", chunk_shift=6,
                                     coarse_chunks=4, batch_products=300000)
    assert info["coarse_rows"] > 0 and info["coarse_shift"] == 8
    # heavy rows' first coarse chunks exceed 1024 products (fine level), the
    # others are sorted directly
    assert 0 < info["coarse_fine_chunks"] < 4 * info["coarse_chunks"]
    compare(rp, col, val, oracle.spgemm(A, A), np.float64, exact=False)
    ctx.set_options(force_category="auto", chunk_shift=0, coarse_chunks=0, batch_products=0)


def test_coarse_chunk_size_boundary(ctx):
    """One row whose coarse chunks (256 columns: chunks of 2^6, 4 per coarse
    chunk) hold exactly 1024 products (sorted directly), 1025 (fine level),
    none, and 1, with repeated columns; the products are a_j * 1 with
    integer a_j, so the sums are exact."""
    rng = np.random.default_rng(93)
    parts = [rng.integers(0, 256, 1024), rng.integers(256, 512, 1025),
             np.array([1023]), rng.integers(1024, 1280, 700)]
    cols = np.concatenate(parts)
    n = len(cols)
    a = rng.integers(-4, 5, n).astype(np.float64)
    A = CSR(2, n, np.array([0, n, n], np.int64), np.arange(n, dtype=np.int32), a)
    B = CSR(n, 1280, np.arange(n + 1, dtype=np.int64), cols.astype(np.int32), np.ones(n))
    log("coarse chunk size boundary")
    rp, col, val, info = gpu_product(ctx, A, B, force_category="chunked", chunk_shift=6,
                                     coarse_chunks=4)
    assert info["coarse_rows"] == 1 and info["coarse_chunks"] == 5
    assert info["coarse_fine_chunks"] == 4  # only the 1025-product coarse chunk
    compare(rp, col, val, oracle.spgemm(A, B), np.float64, exact=True)
    ctx.set_options(force_category="auto", chunk_shift=0, coarse_chunks=0)


@pytest.mark.parametrize("cit", [np.int32, np.int64])
def test_coarse_level_int_values(ctx, cit):
    """Integer-valued products through the coarse level are bit-exact, with
    32- and 64-bit column indices."""
    A = wl.erdos_renyi(700, 900, 9, wl.seed(90), val_kind="int", col_dtype=cit)
    B = wl.erdos_renyi(900, 1 << 17, 60, wl.seed(91), val_kind="int", col_dtype=cit)
    log(f"coarse int col={cit.__name__}")
    rp, col, val, info = gpu_product(ctx, A, B, force_category="chunked", chunk_shift=8,
                                     coarse_chunks=16)
    assert info["coarse_rows"] > 0
    compare(rp, col, val, oracle.spgemm(A, B), np.float64, exact=True)
    ctx.set_options(force_category="auto", chunk_shift=0, coarse_chunks=0)


@pytest.mark.parametrize("rpt", [np.int32, np.int64])
@pytest.mark.parametrize("cit", [np.int32, np.int64])
@pytest.mark.parametrize("vt", [np.float32, np.float64])
def test_index_and_value_types(ctx, rpt, cit, vt):
    A = wl.erdos_renyi(700, 900, 9, wl.seed(82), val_kind="int", val_dtype=vt, rowptr_dtype=rpt,
                       col_dtype=cit)
    B = wl.erdos_renyi(900, 1 << 15, 30, wl.seed(83), val_kind="int", val_dtype=vt,
                       rowptr_dtype=rpt, col_dtype=cit)
    log(f"types rp={rpt.__name__} col={cit.__name__} v={vt.__name__}")
    for cat in CATS:
        rp, col, val, info = gpu_product(ctx, A, B, force_category=cat)
        compare(rp, col, val, oracle.spgemm(A, B), vt, exact=True)
    ctx.set_options(force_category="auto")


def test_banded(ctx):
    A = wl.banded(20000, 64, 8, wl.seed(84))
    log("banded")
    for cat in CATS:
        rp, col, val, info = gpu_product(ctx, A, A, force_category=cat)
        compare(rp, col, val, oracle.spgemm(A, A), np.float64, exact=False)
    ctx.set_options(force_category="auto")


def test_edge_cases(ctx):
    log("edge cases")
    # empty matrix
    E = CSR(0, 5, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    B = wl.erdos_renyi(5, 7, 2, wl.seed(85))
    rp, col, val, info = gpu_product(ctx, E, B)
    assert len(rp) == 1 and rp[0] == 0 and len(col) == 0
    # 1x1
    one = CSR(1, 1, np.array([0, 1]), np.array([0], np.int32), np.array([3.0]))
    rp, col, val, info = gpu_product(ctx, one, one)
    assert list(rp) == [0, 1] and list(col) == [0] and list(val) == [9.0]
    # cancellation to zero is kept; -0.0 becomes +0.0
    A = CSR(2, 2, np.array([0, 2, 3]), np.array([0, 1, 0], np.int32), np.array([1.0, 1.0, 1.0]))
    Bm = CSR(2, 1, np.array([0, 1, 2]), np.array([0, 0], np.int32), np.array([2.0, -2.0]))
    for cat in CATS:
        rp, col, val, info = gpu_product(ctx, A, Bm, force_category=cat)
        assert list(rp) == [0, 1, 2] and list(col) == [0, 0]
        assert val[0] == 0.0 and not np.signbit(val[0]) and val[1] == 2.0
    Bz = CSR(2, 1, np.array([0, 1, 2]), np.array([0, 0], np.int32), np.array([-0.0, -0.0]))
    for cat in CATS:
        rp, col, val, info = gpu_product(ctx, A, Bz, force_category=cat)
        assert not np.signbit(val).any()
    ctx.set_options(force_category="auto")
    # empty rows in A, rows of B that are empty, non-square
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
    for cat in CATS:
        rp, col, val, info = gpu_product(ctx, A2, B2, force_category=cat)
        compare(rp, col, val, oracle.spgemm(A2, B2), np.float64, exact=False)
    ctx.set_options(force_category="auto")


def test_chunk_boundary_columns(ctx):
    """Columns at k*chunkLen - 1 and k*chunkLen, several chunk lengths."""
    log("chunk boundaries")
    for shift in (8, 10, 13):
        L = 1 << shift
        cols = sorted({c for k in range(1, 9) for c in (k * L - 1, k * L, k * L + 1)})
        m = 9 * L + 5
        rows = 64
        A = wl.erdos_renyi(rows, 40, 40, wl.seed(88), val_kind="int")
        # every B row holds all boundary columns
        rpB = np.arange(41, dtype=np.int64) * len(cols)
        colB = np.tile(np.array(cols, np.int32), 40)
        valB = wl.values(len(colB), wl.seed(89), "int", np.float64)
        B = CSR(40, m, rpB, colB, valB)
        for cat in CATS:
            rp, col, val, info = gpu_product(ctx, A, B, force_category=cat, chunk_shift=shift)
            compare(rp, col, val, oracle.spgemm(A, B), np.float64, exact=True)
    ctx.set_options(force_category="auto", chunk_shift=0)


def test_shape_and_type_errors(ctx):
    import paper_2501_07056_amd as mg
    A = wl.erdos_renyi(10, 6, 2, wl.seed(90))
    B = wl.erdos_renyi(7, 6, 2, wl.seed(91))
    dA, dB = mg.DeviceCSR.from_host(A), mg.DeviceCSR.from_host(B)
    with pytest.raises(mg.MagnusError) as e:
        ctx.plan(dA, dB)
    assert e.value.name == "MAGNUS_ERR_SHAPE"
    B2 = wl.erdos_renyi(6, 6, 2, wl.seed(92), val_dtype=np.float32)
    with pytest.raises(mg.MagnusError) as e:
        ctx.plan(dA, mg.DeviceCSR.from_host(B2))
    assert e.value.name == "MAGNUS_ERR_DTYPE"


def test_capacity_error(ctx):
    import torch

    import paper_2501_07056_amd as mg
    A = wl.erdos_renyi(100, 100, 5, wl.seed(93))
    dA = mg.DeviceCSR.from_host(A)
    p = ctx.plan(dA, dA)
    C = p.alloc_output(torch.int64, capacity=p.nnz - 1)
    with pytest.raises(mg.MagnusError) as e:
        p.execute(C)
    assert e.value.name == "MAGNUS_ERR_CAPACITY"
    p.destroy()


def test_row_ip_and_scan(ctx):
    import torch

    import paper_2501_07056_amd as mg
    A, _ = wl.config2(12)
    dA = mg.DeviceCSR.from_host(A)
    ip, tot = ctx.row_ip(dA, dA)
    ref = oracle.ip(A, A)
    assert np.array_equal(ip.cpu().numpy(), ref) and tot == ref.sum()
    x = torch.randint(0, 1 << 40, (3_000_001,), dtype=torch.int64, device="cuda")
    out, total = ctx.exclusive_scan(x)
    xc = x.cpu()
    want = torch.cumsum(xc, 0) - xc
    assert torch.equal(out.cpu(), want) and total == int(xc.sum())
