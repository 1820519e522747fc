"""Pins of the oracle's coarse level (Section 3.3, Algorithm 4) to facts that
do not come from it: brute-force enumeration of the intermediate product,
scipy's CSC conversion, the C++ oracle's per-row product counts, and the
plain product (Eq. 1) for the complete two-level path."""
import numpy as np
import scipy.sparse as sp

import oracle
import workloads as wl
from oracle import coarse


def _brute_products(A, B, i):
    """(j, position in B, column, a*b) of every product of row i, in A's
    entry order then B's."""
    rp, bp = A.rowptr.astype(np.int64), B.rowptr.astype(np.int64)
    out = []
    for p in range(int(rp[i]), int(rp[i + 1])):
        j, a = int(A.col[p]), float(A.val[p])
        for q in range(int(bp[j]), int(bp[j + 1])):
            out.append((j, q, int(B.col[q]), a * float(B.val[q])))
    return out


def _pair(seed, n=40, k=60, m=1 << 12, da=5, db=30, kind="uniform"):
    A = wl.erdos_renyi(n, k, da, wl.seed(seed), val_kind=kind)
    B = wl.erdos_renyi(k, m, db, wl.seed(seed + 1), val_kind=kind)
    return A, B


def test_coarse_rows_b_and_csc():
    A, _ = _pair(200)
    rows = [1, 3, 4, 9, 17, 30, 39]
    rp = A.rowptr.astype(np.int64)
    ref = np.unique(np.concatenate([A.col[rp[i]:rp[i + 1]] for i in rows]))
    assert coarse.coarse_rows_b(A, rows) == ref.tolist()
    colptr, hrow, hval = coarse.csc_of_rows(A, rows)
    S = sp.csr_matrix((A.val, A.col.astype(np.int64), rp), shape=(A.nrows, A.ncols))[rows].tocsc()
    S.sort_indices()
    assert np.array_equal(colptr, S.indptr)
    assert np.array_equal(hrow, S.indices)
    assert np.allclose(hval, S.data, rtol=0, atol=0)


def test_coarse_chunks_hold_each_rows_products_in_outer_product_order():
    A, B = _pair(202)
    rows = [0, 2, 5, 6, 11, 23, 38]
    cs = 9
    off, colc, valc, nc = coarse.coarse_level(A, B, rows, cs)
    assert nc == (1 << 12) >> cs
    assert off[0] == 0 and (np.diff(off) >= 0).all()
    # each row's chunks continue from the previous row's: the row starts
    # after the products of the rows before it (counted by the C++ oracle)
    ipr = oracle.ip(A, B)
    assert np.array_equal(off[::nc][:len(rows)], np.concatenate([[0], np.cumsum(ipr[rows])[:-1]]))
    for r, i in enumerate(rows):
        prods = _brute_products(A, B, i)
        for c in range(nc):
            s0, s1 = off[r * nc + c], off[r * nc + c + 1]
            # outer product over A_hat's columns in ascending order: by B row,
            # then B's entry order
            want = sorted([p for p in prods if p[2] >> cs == c], key=lambda p: (p[0], p[1]))
            assert s1 - s0 == len(want)
            assert np.array_equal(colc[s0:s1], np.array([p[2] - (c << cs) for p in want],
                                                        dtype=np.int64))
            assert np.array_equal(valc[s0:s1], np.array([p[3] for p in want]))
    assert (colc >= 0).all() and (colc < (1 << cs)).all()


def test_two_level_equals_the_product_exactly_on_integers():
    A, B = _pair(204, kind="int")
    rows = list(range(0, A.nrows, 3))
    got = coarse.two_level_rows(A, B, rows, 8, 5)
    ref = oracle.spgemm(A, B, np.array(rows))
    for r in range(len(rows)):
        s0, s1 = ref.rowptr[r], ref.rowptr[r + 1]
        assert np.array_equal(got[r][0], ref.col[s0:s1])
        assert np.array_equal(got[r][1], ref.val[s0:s1])


def test_two_level_within_the_error_bound_on_reals():
    A, B = _pair(206, m=1 << 10, db=40)
    rows = [3, 7, 8, 20, 31]
    got = coarse.two_level_rows(A, B, rows, 7, 4)
    ref = oracle.spgemm(A, B, np.array(rows))
    for r in range(len(rows)):
        s0, s1 = ref.rowptr[r], ref.rowptr[r + 1]
        assert np.array_equal(got[r][0], ref.col[s0:s1])
        err = np.abs(got[r][1] - ref.ref[s0:s1])
        assert (err <= 1e-12 * ref.abssum[s0:s1]).all()
