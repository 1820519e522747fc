"""The seeded generators: determinism, exact structure and distribution."""
import numpy as np
import pytest

import workloads as wl


def test_er_exact_distinct_sorted():
    A = wl.erdos_renyi(2000, 300, 17, wl.seed(50))
    rp = A.rowptr.astype(np.int64)
    assert (np.diff(rp) == 17).all()
    for i in range(A.nrows):
        c = A.col[rp[i]:rp[i + 1]]
        assert (np.diff(c) > 0).all() and c.min() >= 0 and c.max() < 300


def test_er_deterministic_and_thread_independent():
    A = wl.erdos_renyi(5000, 1 << 20, 16, wl.seed(51))
    B = wl.erdos_renyi(5000, 1 << 20, 16, wl.seed(51))
    assert (A.col == B.col).all() and (A.val == B.val).all()
    rp = np.empty(5001, dtype=np.int64)
    col = np.empty(5000 * 16, dtype=np.int32)
    wl._load().wl_er(5000, 1 << 20, 16, wl.seed(51), wl._ptr(rp), wl._ptr(col), 4, 1)
    assert (col == A.col).all()


def test_er_uniform_columns():
    A = wl.erdos_renyi(20000, 64, 8, wl.seed(52))
    h = np.bincount(A.col, minlength=64)
    exp = A.nnz / 64
    assert np.abs(h - exp).max() < 6 * np.sqrt(exp)


def test_er_wide_rows_mask_and_threads():
    """Wide rows: exactly d distinct sorted columns in [0, m) in the rows the
    mask names, empty rows elsewhere, the same for any thread count, and
    uniform columns (also where m is only 2d and duplicates are common)."""
    n, m, d = 3000, 1 << 12, 300
    mask = (np.arange(n) % 3 != 1).astype(np.uint8)
    A = wl.erdos_renyi_wide(n, m, d, wl.seed(55), rows_mask=mask)
    rp = A.rowptr.astype(np.int64)
    assert (np.diff(rp) == d * mask.astype(np.int64)).all()
    for i in range(0, n, 7):
        c = A.col[rp[i]:rp[i + 1]]
        assert (np.diff(c) > 0).all() and (len(c) == 0 or (c.min() >= 0 and c.max() < m))
    rp1 = np.empty(n + 1, dtype=np.int64)
    col1 = np.empty(A.nnz, dtype=np.int32)
    assert wl._load().wl_er_wide(n, m, d, wl.seed(55), wl._ptr(mask), wl._ptr(rp1),
                                 wl._ptr(col1), 4, 1) == A.nnz
    assert (col1 == A.col).all() and (rp1 == rp).all()
    h = np.bincount(A.col, minlength=m)
    exp = A.nnz / m
    assert np.abs(h - exp).max() < 6 * np.sqrt(exp)
    B = wl.erdos_renyi_wide(500, 2 * 400, 400, wl.seed(56))
    rb = B.rowptr.astype(np.int64)
    assert all(len(np.unique(B.col[rb[i]:rb[i + 1]])) == 400 for i in range(500))
    with pytest.raises(ValueError):
        wl.erdos_renyi_wide(10, 100, 60, wl.seed(57))


def test_massive_er_shape():
    A, B = wl.massive_er(20, d=32, nrows=64)
    assert A.nrows == 64 and A.ncols == 64 * 32 == B.nrows and B.ncols == 1 << 20
    assert (np.diff(A.rowptr) == 32).all()
    ref = np.zeros(B.nrows, bool)
    ref[A.col] = True
    assert np.array_equal(np.diff(B.rowptr) > 0, ref)
    assert (np.diff(B.rowptr)[ref] == 32).all()
    assert A.val.dtype == np.float32 and B.col.dtype == np.int32


def test_banded_constraint():
    B = wl.banded(3000, 64, 8, wl.seed(53))
    rp = B.rowptr.astype(np.int64)
    assert (np.diff(rp) == 9).all()
    for i in range(B.nrows):
        c = B.col[rp[i]:rp[i + 1]].astype(np.int64)
        assert (np.diff(c) > 0).all()
        assert i in c
        assert (np.abs(c - i) <= 64).all()


def test_rmat_quadrant_frequencies():
    # before merging, every level of every draw picks quadrant (0,0),(0,1),(1,0),(1,1)
    # with probability a, b, c, d = .57, .19, .19, .05
    s = 14
    R = wl.rmat(s, wl.seed(54), merge=False)
    rows = np.repeat(np.arange(R.nrows), np.diff(R.rowptr.astype(np.int64)))
    cols = R.col.astype(np.int64)
    assert R.nnz == 16 << s
    for lvl in (s - 1, s // 2, 0):
        rb = (rows >> lvl) & 1
        cb = (cols >> lvl) & 1
        freq = np.array([np.mean((rb == 0) & (cb == 0)), np.mean((rb == 0) & (cb == 1)),
                         np.mean((rb == 1) & (cb == 0)), np.mean((rb == 1) & (cb == 1))])
        assert np.allclose(freq, [0.57, 0.19, 0.19, 0.05], atol=0.005), freq


def test_rmat_merge_removes_only_duplicates():
    U = wl.rmat(12, wl.seed(55), merge=False)
    M = wl.rmat(12, wl.seed(55))
    ru, rm = U.rowptr.astype(np.int64), M.rowptr.astype(np.int64)
    for i in range(0, U.nrows, 37):
        assert np.array_equal(np.unique(U.col[ru[i]:ru[i + 1]]), M.col[rm[i]:rm[i + 1]])


def test_values_ranges():
    v = wl.values(100000, wl.seed(56), "uniform", np.float64)
    assert v.min() >= -1 and v.max() < 1 and abs(v.mean()) < 0.01
    f = wl.values(100000, wl.seed(56), "uniform", np.float32)
    assert f.dtype == np.float32 and f.min() >= -1 and f.max() < 1
    k = wl.values(90000, wl.seed(57), "int", np.float64)
    assert set(np.unique(k).tolist()) == set(range(-4, 5))


def test_config4_shapes_ranges():
    sh = wl.config4_shapes()
    assert len(sh) == 512
    ns = np.array([s[0] for s in sh])
    ds = np.array([s[1] for s in sh])
    assert ns.min() >= 1024 and ns.max() <= 65536 and ds.min() >= 4 and ds.max() <= 32
    # log-uniform: the median of log n is near the middle of [ln 1024, ln 65536]
    assert abs(np.median(np.log(ns)) - 0.5 * (np.log(1024) + np.log(65536))) < 0.3


def test_config5_stream():
    reqs = wl.config5_requests(400, qps=5.0)
    gaps = np.diff([0.0] + [r.arrival_s for r in reqs])
    assert abs(gaps.mean() - 0.2) < 0.05
    kinds = [r.kind for r in reqs]
    assert 0.4 < kinds.count("rmat") / len(kinds) < 0.6
    for r in reqs:
        if r.kind == "rmat":
            assert r.n & (r.n - 1) == 0


def test_autotune_size_class_keys():
    """Size classes group products by value type, rows and row lengths."""
    import importlib
    at = importlib.import_module("paper_2501_07056_amd.autotune")
    A = wl.erdos_renyi(1000, 1000, 8, wl.seed(50), val_dtype=np.float32)
    B = wl.erdos_renyi(1000, 1000, 30, wl.seed(51), val_dtype=np.float64)
    assert at.size_class(A, A) == "f32/n10/da3/db3"
    assert at.size_class(B, B) == "f64/n10/da5/db5"
    assert at.size_class(A, B) == "f32/n10/da3/db5"
