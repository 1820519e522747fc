"""CHUNKED rows binned by runs (GPU): the part of each B row inside one column
chunk is reordered as a whole, and every chunk's accumulator reads its
products from B through its list of runs (options.chunk_runs = 1 forces it,
0 lets the plan choose).  Each case compares with the oracle element by
element: structure exactly, values bit-exactly on integer data and within
rtol * sum|a_ik b_kj| otherwise."""
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


def _runs(ctx, A, B, vt, exact, rowptr_dtype="int64", **opts):
    rp, col, val, info = gpu_product(ctx, A, B, rowptr_dtype=rowptr_dtype, chunk_runs=1,
                                     force_category="chunked", **opts)
    assert info["run_binned"] == 1 and info["n_runs"] > 0, info
    compare(rp, col, val, oracle.spgemm(A, B), vt, exact=exact)
    ctx.set_options(chunk_runs=0, force_category="auto", chunk_shift=0, bin_dense_min=0,
                    sort_group_max=0, dense_block=0)
    return info


@pytest.mark.parametrize("shift", [13, 9, 6])
def test_runs_rmat(ctx, shift):
    """Power-law rows: long runs in the heavy B rows; chunk lengths from the
    default down to 64 columns (many chunks per row, dense and sorted
    chunks)."""
    A, _ = wl.config2(12)
    log(f"runs rmat12 shift={shift}")
    info = _runs(ctx, A, A, np.float64, False, chunk_shift=shift)
    assert info["n_runs"] < info["ip_by_category"][2]


def test_runs_rmat_integer_exact(ctx):
    A, _ = wl.config2(12)
    Ai = CSR(A.nrows, A.ncols, A.rowptr, A.col, wl.values(A.nnz, wl.seed(120), "int", np.float64))
    log("runs rmat12 integer")
    for dmin, gmax in ((0, 0), (64, 32), (1025, 1024)):
        _runs(ctx, Ai, Ai, np.float64, True, chunk_shift=8, bin_dense_min=dmin,
              sort_group_max=gmax)


@pytest.mark.parametrize("vt", [np.float64, np.float32])
def test_runs_er(ctx, vt):
    A = wl.erdos_renyi(3000, 5000, 12, wl.seed(121), val_dtype=vt)
    B = wl.erdos_renyi(5000, 20000, 20, wl.seed(122), val_dtype=vt)
    log(f"runs er vt={vt.__name__}")
    _runs(ctx, A, B, vt, False)
    _runs(ctx, A, B, vt, False, chunk_shift=8)


@pytest.mark.parametrize("rpt", [np.int32, np.int64])
@pytest.mark.parametrize("cit", [np.int32, np.int64])
@pytest.mark.parametrize("vt", [np.float32, np.float64])
def test_runs_index_and_value_types(ctx, rpt, cit, vt):
    A = wl.erdos_renyi(700, 900, 9, wl.seed(123), val_kind="int", val_dtype=vt, rowptr_dtype=rpt,
                       col_dtype=cit)
    B = wl.erdos_renyi(900, 1 << 15, 30, wl.seed(124), val_kind="int", val_dtype=vt,
                       rowptr_dtype=rpt, col_dtype=cit)
    log(f"runs types rp={rpt.__name__} col={cit.__name__} v={vt.__name__}")
    _runs(ctx, A, B, vt, True, chunk_shift=10)
    _runs(ctx, A, B, vt, True, rowptr_dtype="int32", chunk_shift=10)


def test_runs_dense_block_sizes(ctx):
    A, _ = wl.config2(11)
    Ai = CSR(A.nrows, A.ncols, A.rowptr, A.col, wl.values(A.nnz, wl.seed(125), "int", np.float64))
    for blk in (256, 512, 1024):
        log(f"runs dense block {blk}")
        _runs(ctx, Ai, Ai, np.float64, True, chunk_shift=7, dense_block=blk, bin_dense_min=16)


def test_runs_chunk_boundaries_and_thresholds(ctx):
    """Runs that end at k*chunkLen - 1 and start at k*chunkLen; one row whose
    chunks hold 511, 1, 2, 512, 513, 1023, 1024, 1025, 0 and 1 products,
    gathered from runs of a few long B rows."""
    log("runs boundaries")
    for shift in (8, 10, 13):
        L = 1 << shift
        cols = sorted({c for k in range(1, 9) for c in (k * L - 1, k * L, k * L + 1)})
        A = wl.erdos_renyi(64, 40, 40, wl.seed(126), val_kind="int")
        rpB = np.arange(41, dtype=np.int64) * len(cols)
        colB = np.tile(np.array(cols, np.int32), 40)
        B = CSR(40, 9 * L + 5, rpB, colB, wl.values(len(colB), wl.seed(127), "int", np.float64))
        _runs(ctx, A, B, np.float64, True, chunk_shift=shift)
    # chunk product counts at the accumulator thresholds: row 0 of A has
    # eight entries, B rows 0..7 split each chunk's columns among them
    L = 1 << 11
    counts = [511, 1, 2, 512, 513, 1023, 1024, 1025, 0, 1]
    rng = np.random.default_rng(128)
    rows = [[] for _ in range(8)]
    for c, k in enumerate(counts):
        cols = np.sort(rng.choice(L, k, replace=False)) + c * L
        for r, part in enumerate(np.array_split(cols, 8)):
            rows[r].extend(part.tolist())
    # B rows need distinct ascending columns: the split keeps each part sorted
    rpB = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    B = CSR(8, len(counts) * L, rpB, np.concatenate([np.array(r, np.int32) for r in rows]),
            rng.integers(-4, 5, int(rpB[-1])).astype(np.float64))
    A = CSR(2, 8, np.array([0, 8, 8], np.int64), np.arange(8, dtype=np.int32),
            rng.integers(1, 5, 8).astype(np.float64))
    # sorted chunks packed up to 512 products: {511, 1}, {2}, {512}, {513},
    # {1023}, {1}; then the default packing (up to 1024 products)
    info = _runs(ctx, A, B, np.float64, True, chunk_shift=11, sort_group_max=512)
    assert info["n_dense_chunks"] == 2 and info["n_sort_groups"] == 6
    assert info["n_bins"] == len(counts)
    info = _runs(ctx, A, B, np.float64, True, chunk_shift=11)
    assert info["n_dense_chunks"] == 2 and info["n_bins"] == len(counts)


def test_runs_edge_cases(ctx):
    log("runs edge cases")
    # empty rows of A and of B, non-square
    A = wl.erdos_renyi(400, 300, 5, wl.seed(129), val_kind="int")
    rpA = A.rowptr.astype(np.int64)
    keep = np.ones(A.nnz, bool)
    for i in range(0, 400, 7):
        keep[rpA[i]:rpA[i + 1]] = False
    cnt = np.array([keep[rpA[i]:rpA[i + 1]].sum() for i in range(400)])
    A2 = CSR(400, 300, np.concatenate([[0], np.cumsum(cnt)]), A.col[keep], A.val[keep])
    Bs = wl.erdos_renyi(300, 50000, 40, wl.seed(130), val_kind="int")
    rpB = Bs.rowptr.astype(np.int64)
    keepB = np.ones(Bs.nnz, bool)
    for j in range(0, 300, 5):
        keepB[rpB[j]:rpB[j + 1]] = False
    cntB = np.array([keepB[rpB[j]:rpB[j + 1]].sum() for j in range(300)])
    B2 = CSR(300, 50000, np.concatenate([[0], np.cumsum(cntB)]), Bs.col[keepB], Bs.val[keepB])
    _runs(ctx, A2, B2, np.float64, True, chunk_shift=9)
    # cancellation to zero is kept and is +0.0
    A = CSR(2, 2, np.array([0, 2, 3]), np.array([0, 1, 0], np.int32), np.array([1.0, 1.0, 1.0]))
    Bm = CSR(2, 40000, np.array([0, 2, 4]), np.array([0, 30000, 0, 30000], np.int32),
             np.array([2.0, -0.0, -2.0, -0.0]))
    rp, col, val, info = gpu_product(ctx, A, Bm, chunk_runs=1, force_category="chunked",
                                     chunk_shift=8)
    assert info["run_binned"] == 1
    assert list(rp) == [0, 2, 4] and list(col) == [0, 30000, 0, 30000]
    assert val[0] == 0.0 and not np.signbit(val).any()
    ctx.set_options(chunk_runs=0, force_category="auto", chunk_shift=0)


def _runs_and_products(A, B, shift):
    """Runs (distinct chunks of each referenced B row, over A's entries) and
    products of C = A*B with chunks of 2^shift columns (host count)."""
    rpB = B.rowptr.astype(np.int64)
    ch = B.col.astype(np.int64) >> shift
    nseg = np.zeros(B.nrows, np.int64)
    for j in range(B.nrows):
        nseg[j] = len(np.unique(ch[rpB[j]:rpB[j + 1]]))
    blen = np.diff(rpB)
    acol = A.col.astype(np.int64)
    return int(nseg[acol].sum()), int(blen[acol].sum())


def test_runs_auto_choice(ctx):
    """chunk_runs = 0: runs where the rows hold at least 8 products per run,
    single products below; -1 never uses runs."""
    log("runs auto choice")
    cases = [
        # long B rows over few chunks: many products per run
        (wl.erdos_renyi(300, 400, 8, wl.seed(133)), wl.erdos_renyi(400, 1 << 14, 200, wl.seed(134)), 11),
        # B rows spread over a wide range: about one product per run
        (wl.erdos_renyi(500, 600, 16, wl.seed(131)), wl.erdos_renyi(600, 1 << 20, 16, wl.seed(132)), 10),
    ]
    for A, B, shift in cases:
        runs, prods = _runs_and_products(A, B, shift)
        want = 1 if prods >= 8 * runs else 0
        rp, col, val, info = gpu_product(ctx, A, B, force_category="chunked", chunk_shift=shift)
        assert info["run_binned"] == want, (runs, prods, info["run_binned"])
        if want:
            assert info["n_runs"] == runs
        ref = oracle.spgemm(A, B)
        compare(rp, col, val, ref, np.float64, exact=False)
        rp, col, val, info = gpu_product(ctx, A, B, force_category="chunked", chunk_shift=shift,
                                         chunk_runs=-1)
        assert info["run_binned"] == 0
        compare(rp, col, val, ref, np.float64, exact=False)
        ctx.set_options(chunk_runs=0)
    ctx.set_options(chunk_runs=0, force_category="auto", chunk_shift=0)
