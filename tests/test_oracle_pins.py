"""Pins of the CPU oracle to facts that do not come from the oracle itself:
dense and boolean matrix products, closed forms (identity, permutations,
power-of-two diagonals), structural identities, scipy's sparse product,
exact rational sums, and error bounds.

The oracle computes Gustavson's formula (Section 2.1, Eq. 1) with the dense
accumulator's semantics (Algorithm 1: slots start at +0.0, structural entries
are kept whatever their value)."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as wl
from workloads import CSR


def csr_from_dense(D, rp=np.int64, ci=np.int32, vt=np.float64, keep=None):
    """CSR of the entries where keep (default D != 0) holds, columns ascending."""
    keep = (D != 0) if keep is None else keep
    n, m = D.shape
    rowptr = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for i in range(n):
        js = np.nonzero(keep[i])[0]
        cols.extend(js.tolist())
        vals.extend(D[i, js].tolist())
        rowptr[i + 1] = rowptr[i] + len(js)
    return CSR(n, m, rowptr.astype(rp), np.array(cols, dtype=ci), np.array(vals, dtype=vt))


def to_scipy(A):
    return sp.csr_matrix((A.val.astype(np.float64), A.col.astype(np.int64),
                          A.rowptr.astype(np.int64)), shape=(A.nrows, A.ncols))


def from_scipy(S, vt=np.float64):
    S = sp.csr_matrix(S)
    S.sort_indices()
    return CSR(S.shape[0], S.shape[1], S.indptr.astype(np.int64), S.indices.astype(np.int64),
               S.data.astype(vt))


def dense_of(r, n, m):
    D = np.zeros((n, m))
    P = np.zeros((n, m), dtype=bool)
    for k, i in enumerate(r.rows):
        for p in range(r.rowptr[k], r.rowptr[k + 1]):
            D[i, r.col[p]] = r.val[p]
            P[i, r.col[p]] = True
    return D, P


def rand_int_sparse(rng, n, m, density, lo=-4, hi=4):
    D = rng.integers(lo, hi + 1, size=(n, m)).astype(np.float64)
    keep = rng.random((n, m)) < density
    return D * keep, keep


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 7, 3), (17, 9, 23), (40, 40, 40), (3, 60, 2)])
def test_dense_and_boolean_products(shape):
    rng = np.random.default_rng(7 + sum(shape))
    n, k, m = shape
    DA, KA = rand_int_sparse(rng, n, k, 0.3)
    DB, KB = rand_int_sparse(rng, k, m, 0.3)
    A = csr_from_dense(DA, keep=KA)
    B = csr_from_dense(DB, keep=KB)
    r = oracle.spgemm(A, B)
    D, P = dense_of(r, n, m)
    # values: the textbook dense product (exact for these small integers)
    assert np.array_equal(D, DA @ DB)
    # structure: the boolean product of the stored patterns
    assert np.array_equal(P, (KA.astype(np.int64) @ KB.astype(np.int64)) > 0)
    # the input-precision sum equals the high-precision one on exact data
    assert np.array_equal(r.val, r.ref)


def test_exhaustive_3x3_patterns():
    """Every pair of 3x3 patterns, as one block-diagonal product."""
    pats = np.array([[(p >> b) & 1 for b in range(9)] for p in range(512)], dtype=bool)
    pats = pats.reshape(512, 3, 3)
    idx = np.arange(9).reshape(3, 3)
    va = (1 + idx).astype(np.float64)                        # 1..9
    vb = np.where((idx % 2) == 0, 1.0, -2.0) * (1 + idx % 3)  # mixed signs -> cancellations
    K = 512 * 512
    pa = np.repeat(np.arange(512), 512)
    pb = np.tile(np.arange(512), 512)

    def block_diag(which, vals):
        keep = pats[which]                               # K x 3 x 3
        rows = np.repeat(np.arange(3 * K), 3).reshape(K, 3, 3)
        cols = (3 * np.arange(K))[:, None, None] + np.arange(3)[None, None, :]
        cols = np.broadcast_to(cols, (K, 3, 3))
        v = np.broadcast_to(vals, (K, 3, 3))
        r, c, x = rows[keep], cols[keep], v[keep]
        counts = np.bincount(r, minlength=3 * K)
        rp = np.concatenate([[0], np.cumsum(counts)])
        return CSR(3 * K, 3 * K, rp.astype(np.int64), c.astype(np.int32), x.astype(np.float64))

    A = block_diag(pa, va)
    B = block_diag(pb, vb)
    r = oracle.spgemm(A, B)
    DA = pats[pa] * va
    DB = pats[pb] * vb
    DC = np.einsum("kij,kjl->kil", DA, DB)
    PC = np.einsum("kij,kjl->kil", pats[pa].astype(np.int64), pats[pb].astype(np.int64)) > 0
    # scatter the oracle output back into K 3x3 blocks
    rows = np.repeat(np.arange(3 * K), np.diff(r.rowptr))
    blk = rows // 3
    assert (r.col // 3 == blk).all()
    gotP = np.zeros((K, 3, 3), dtype=bool)
    gotV = np.zeros((K, 3, 3))
    gotP[blk, rows % 3, r.col % 3] = True
    gotV[blk, rows % 3, r.col % 3] = r.val
    assert np.array_equal(gotP, PC)
    assert np.array_equal(gotV, DC)
    # structural zeros from cancellation are kept
    assert ((DC == 0) & PC).sum() > 0


# ---------------------------------------------------------------- closed forms
def _rand_csr(seed_, n, m, d, vt=np.float64, kind="uniform"):
    return wl.erdos_renyi(n, m, d, seed_, val_kind=kind, val_dtype=vt)


def _identity(n, vt=np.float64):
    return CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
               np.ones(n, dtype=vt))


def _same(r, M):
    assert np.array_equal(r.rowptr, M.rowptr.astype(np.int64))
    assert np.array_equal(r.col, M.col.astype(np.int64))
    assert np.array_equal(r.val, M.val.astype(np.float64))


@pytest.mark.parametrize("vt", [np.float64, np.float32])
def test_identity_products(vt):
    A = _rand_csr(wl.seed(60), 300, 500, 9, vt)
    _same(oracle.spgemm(A, _identity(500, vt)), A)
    _same(oracle.spgemm(_identity(300, vt), A), A)


def test_permutation_products():
    rng = np.random.default_rng(3)
    A = _rand_csr(wl.seed(61), 200, 200, 7)
    perm = rng.permutation(200)
    # P has P[i, perm[i]] = 1, so (P A) row i = A row perm[i]
    P = CSR(200, 200, np.arange(201, dtype=np.int64), perm.astype(np.int32), np.ones(200))
    r = oracle.spgemm(P, A)
    rp = A.rowptr.astype(np.int64)
    for i in range(200):
        j = perm[i]
        assert np.array_equal(r.col[r.rowptr[i]:r.rowptr[i + 1]], A.col[rp[j]:rp[j + 1]])
        assert np.array_equal(r.val[r.rowptr[i]:r.rowptr[i + 1]], A.val[rp[j]:rp[j + 1]])
    # (A P)[i, perm[k]] = A[i, k]: column k of A moves to column perm[k]
    r2 = oracle.spgemm(A, P.astype(val=np.float64))
    for i in range(200):
        got = dict(zip(r2.col[r2.rowptr[i]:r2.rowptr[i + 1]].tolist(),
                       r2.val[r2.rowptr[i]:r2.rowptr[i + 1]].tolist()))
        want = {int(perm[c]): float(v) for c, v in zip(A.col[rp[i]:rp[i + 1]], A.val[rp[i]:rp[i + 1]])}
        assert got == want


def test_power_of_two_diagonal_scales_exactly():
    A = _rand_csr(wl.seed(62), 150, 90, 11)
    e = np.arange(150) % 7 - 3
    D = CSR(150, 150, np.arange(151, dtype=np.int64), np.arange(150, dtype=np.int32),
            np.ldexp(1.0, e))
    r = oracle.spgemm(D, A)
    rp = A.rowptr.astype(np.int64)
    assert np.array_equal(r.col, A.col.astype(np.int64))
    want = np.concatenate([np.ldexp(A.val[rp[i]:rp[i + 1]], e[i]) for i in range(150)])
    assert np.array_equal(r.val, want)


def test_zero_row_and_empty_matrix():
    A = _rand_csr(wl.seed(63), 50, 60, 5)
    rp = A.rowptr.astype(np.int64).copy()
    # empty out row 10 of A
    cut = rp[11] - rp[10]
    col = np.delete(A.col, np.arange(rp[10], rp[11]))
    val = np.delete(A.val, np.arange(rp[10], rp[11]))
    rp[11:] -= cut
    A2 = CSR(50, 60, rp, col, val)
    B = _rand_csr(wl.seed(64), 60, 40, 4)
    r = oracle.spgemm(A2, B)
    assert r.rowptr[11] == r.rowptr[10]
    E = CSR(0, 60, np.zeros(1, dtype=np.int64), np.zeros(0, np.int32), np.zeros(0))
    r0 = oracle.spgemm(E, B)
    assert r0.nnz == 0 and len(r0.rowptr) == 1


def test_cancellation_and_signed_zero():
    # 1*2 + 1*(-2) = 0: the entry is kept and is +0.0 (slots start at +0.0)
    A = CSR(1, 2, np.array([0, 2]), np.array([0, 1], np.int32), np.array([1.0, 1.0]))
    B = CSR(2, 1, np.array([0, 1, 2]), np.array([0, 0], np.int32), np.array([2.0, -2.0]))
    r = oracle.spgemm(A, B)
    assert r.nnz == 1 and r.val[0] == 0.0 and not np.signbit(r.val[0])
    # a single -0.0 product: +0.0 + (-0.0) = +0.0
    A = CSR(1, 1, np.array([0, 1]), np.array([0], np.int32), np.array([1.0]))
    B = CSR(1, 1, np.array([0, 1]), np.array([0], np.int32), np.array([-0.0]))
    r = oracle.spgemm(A, B)
    assert r.nnz == 1 and not np.signbit(r.val[0]) and not np.signbit(r.ref[0])
    for vt in (np.float32,):
        r = oracle.spgemm(A.astype(val=vt), B.astype(val=vt))
        assert not np.signbit(r.val[0])


def test_shape_mismatch_rejected():
    A = _rand_csr(wl.seed(65), 5, 6, 2)
    B = _rand_csr(wl.seed(66), 7, 6, 2)
    with pytest.raises(ValueError):
        oracle.spgemm(A, B)


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("which", ["er", "rmat", "banded"])
def test_structural_invariants(which):
    if which == "er":
        A = _rand_csr(wl.seed(67), 700, 700, 12)
        B = A
    elif which == "rmat":
        A = wl.rmat(10, wl.seed(68))
        B = A
    else:
        A = wl.banded(900, 64, 8, wl.seed(69))
        B = A
    r = oracle.spgemm(A, B)
    m = B.ncols
    assert (np.diff(r.rowptr) >= 0).all() and r.rowptr[-1] == len(r.col)
    ipr = oracle.ip(A, B)
    # two independent counts of the intermediate product (Section 4.3):
    # per row, and as sum_j colcount_A(j) * rowlen_B(j)
    cc = np.bincount(A.col.astype(np.int64), minlength=A.ncols)
    rl = np.diff(B.rowptr.astype(np.int64))
    assert ipr.sum() == int((cc * rl).sum())
    nnzr = np.diff(r.rowptr)
    assert (nnzr <= np.minimum(ipr, m)).all()
    for i in range(A.nrows):
        c = r.col[r.rowptr[i]:r.rowptr[i + 1]]
        assert (np.diff(c) > 0).all()
        if len(c):
            assert c[0] >= 0 and c[-1] < m


def test_transpose_identity():
    """(AB)^T = B^T A^T exactly on integer data (transposes by scipy)."""
    A = _rand_csr(wl.seed(70), 120, 80, 6, kind="int")
    B = _rand_csr(wl.seed(71), 80, 150, 5, kind="int")
    r = oracle.spgemm(A, B)
    C = sp.csr_matrix((r.val, r.col, r.rowptr), shape=(120, 150))
    At = from_scipy(to_scipy(A).T)
    Bt = from_scipy(to_scipy(B).T)
    rt = oracle.spgemm(Bt, At)
    Ct = sp.csr_matrix((rt.val, rt.col, rt.rowptr), shape=(150, 120))
    CT = sp.csr_matrix(C.T)
    CT.sort_indices()
    assert np.array_equal(CT.indptr, Ct.indptr)
    assert np.array_equal(CT.indices, Ct.indices)
    assert np.array_equal(CT.data, Ct.data)


def test_associativity_of_patterns():
    A = _rand_csr(wl.seed(72), 60, 70, 4)
    B = _rand_csr(wl.seed(73), 70, 80, 3)
    Cm = _rand_csr(wl.seed(74), 80, 50, 3)

    def as_csr(r, n, m, vt=np.float64):
        return CSR(n, m, r.rowptr, r.col.astype(np.int64), r.val.astype(vt))

    AB = as_csr(oracle.spgemm(A, B), 60, 80)
    BC = as_csr(oracle.spgemm(B, Cm), 70, 50)
    L = oracle.spgemm(AB, Cm)
    R = oracle.spgemm(A, BC)
    assert np.array_equal(L.rowptr, R.rowptr) and np.array_equal(L.col, R.col)


def test_scipy_agreement():
    """scipy's sparse product (a different summation routine) agrees: path
    counts exactly on all-ones patterns, values within the summation bound."""
    A = wl.rmat(9, wl.seed(75))
    ones = A.astype(val=np.float64)
    ones.val[:] = 1.0
    r1 = oracle.spgemm(ones, ones)
    S = to_scipy(ones) @ to_scipy(ones)
    S.sort_indices()
    assert np.array_equal(S.indptr, r1.rowptr) and np.array_equal(S.indices, r1.col)
    assert np.array_equal(S.data, r1.val)
    r = oracle.spgemm(A, A)
    T = (to_scipy(A) @ to_scipy(A)).tocsr()
    T.sort_indices()
    D, P = dense_of(r, A.nrows, A.ncols)
    Dt = T.toarray()
    ab = np.zeros_like(D)
    for k in range(len(r.rows)):
        ab[k, r.col[r.rowptr[k]:r.rowptr[k + 1]]] = r.abssum[r.rowptr[k]:r.rowptr[k + 1]]
    kmax = int(np.max(oracle.ip(A, A)))
    u = 2.0 ** -53
    assert (np.abs(D - Dt) <= 2 * kmax * u * ab + 1e-300).all()


# ---------------------------------------------------------------- exact sums
@pytest.mark.parametrize("vt", [np.float64, np.float32])
def test_ref_and_val_against_exact_rational_sums(vt):
    A = _rand_csr(wl.seed(76), 40, 30, 6, vt)
    B = _rand_csr(wl.seed(77), 30, 40, 6, vt)
    r = oracle.spgemm(A, B)
    arp, brp = A.rowptr.astype(np.int64), B.rowptr.astype(np.int64)
    u = 2.0 ** -53 if vt == np.float64 else 2.0 ** -24
    for i in range(A.nrows):
        exact = {}
        cnt = {}
        for p in range(arp[i], arp[i + 1]):
            j = int(A.col[p])
            for q in range(brp[j], brp[j + 1]):
                k = int(B.col[q])
                exact[k] = exact.get(k, Fraction(0)) + Fraction(float(A.val[p])) * Fraction(float(B.val[q]))
                cnt[k] = cnt.get(k, 0) + 1
        cols = r.col[r.rowptr[i]:r.rowptr[i + 1]].tolist()
        assert cols == sorted(exact)
        for off, k in enumerate(cols):
            e = float(exact[k])
            ref = r.ref[r.rowptr[i] + off]
            val = r.val[r.rowptr[i] + off]
            ab = r.abssum[r.rowptr[i] + off]
            # long double products and sums: far inside a double ulp of the exact sum
            assert abs(ref - e) <= 2.0 ** -52 * abs(e) + cnt[k] * 2.0 ** -63 * ab
            # the input-precision sum lies within gamma_k of the exact sum
            gam = cnt[k] * u / (1 - cnt[k] * u)
            assert abs(val - e) <= gam * ab * 1.0000001 + 1e-300


# ---------------------------------------------------------------- config closed forms
def test_config1_closed_forms():
    A, B = wl.config1()
    ipr = oracle.ip(A, B)
    assert (ipr == 64).all() and ipr.sum() == 262144
    r = oracle.spgemm(A, B)
    # a row's 64 products come from 8 independent B rows of 8 distinct uniform
    # columns, so a given column is missed with probability (1 - 8/4096)^8:
    # E[nnz per row] = 4096 * (1 - (1 - 1/512)^8) = 63.56
    mean = r.nnz / 4096
    assert abs(mean - 4096 * (1 - (1 - 1 / 512) ** 8)) < 0.05
    assert np.array_equal(r.val, r.ref)  # integer data: every partial sum exact


def test_config3_ip_closed_form_small():
    A, B = wl.config3(logn=12)
    ipr = oracle.ip(A, B)
    assert (ipr == 256).all() and ipr.sum() == 256 << 12


# ---------------------------------------------------------------- val: order and precision
def _col0_chain(vt, bvals, avals=None):
    """A is 1 x k with its entries in stored order on columns 0..k-1; B row j
    holds one entry on column 0 with value bvals[j]: C[0, 0] sums the k
    products a_j * b_j in A's stored order (Algorithm 1's update order)."""
    k = len(bvals)
    avals = [1.0] * k if avals is None else avals
    A = CSR(1, k, np.array([0, k], dtype=np.int64), np.arange(k, dtype=np.int32),
            np.array(avals, dtype=vt))
    B = CSR(k, 1, np.arange(k + 1, dtype=np.int64), np.zeros(k, dtype=np.int32),
            np.array(bvals, dtype=vt))
    return oracle.spgemm(A, B)


def test_val_f64_stored_order_closed_form():
    # products [2^53, 1, -2^53]: (+0 + 2^53) + 1 is a tie between 2^53 and
    # 2^53 + 2 and rounds to even (2^53); minus 2^53 gives 0.  The exact sum
    # (the long double reference) is 1.
    big = 2.0 ** 53
    r = _col0_chain(np.float64, [big, 1.0, -big])
    assert r.val[0] == 0.0 and r.ref[0] == 1.0
    # the reverse storage order: -2^53 + 1 = -(2^53 - 1) is exact, then + 2^53
    r2 = _col0_chain(np.float64, [-big, 1.0, big])
    assert r2.val[0] == 1.0 and r2.ref[0] == 1.0
    # a sum taken in sorted-by-magnitude or any other order would differ from
    # one of the two; the stored order is what decides


def test_val_f32_stored_order_and_input_precision():
    # f32: 2^24 + 1 rounds to 2^24 in single precision, so the stored-order
    # single-precision sum of [2^24, 1, -2^24] is 0; a sum carried in double
    # (then rounded to f32) would give 1, as the double reference does
    big = 2.0 ** 24
    r = _col0_chain(np.float32, [big, 1.0, -big])
    assert r.val[0] == 0.0
    assert r.ref[0] == 1.0
    r2 = _col0_chain(np.float32, [-big, 1.0, big])
    assert r2.val[0] == 1.0


def test_val_products_rounded_before_the_add():
    # f32 products are rounded to single precision before they are added (no
    # fused multiply-add): a = 1 + 2^-12, b = 1 + 2^-12 gives a*b = 1 + 2^-11
    # + 2^-24, which rounds (tie, to even) to 1 + 2^-11 in f32; adding -1
    # then leaves exactly 2^-11.  A fused or double-precision product would
    # keep the 2^-24 term.
    a = 1.0 + 2.0 ** -12
    r = _col0_chain(np.float32, [a, -1.0], avals=[a, 1.0])
    assert r.val[0] == np.float32(2.0 ** -11)
    assert r.ref[0] == 2.0 ** -11 + 2.0 ** -24


def test_val_starts_from_positive_zero():
    # every slot starts at +0.0 (Algorithm 1): a single product -0.0 gives
    # +0.0 + -0.0 = +0.0, and two -0.0 products give +0.0 as well
    for vt in (np.float64, np.float32):
        r = _col0_chain(vt, [-0.0])
        assert r.val[0] == 0.0 and not np.signbit(r.val[0])
        r = _col0_chain(vt, [-0.0, -0.0])
        assert not np.signbit(r.val[0])


@pytest.mark.parametrize("vt", [np.float64, np.float32])
def test_val_random_matches_stored_order_loop(vt):
    # a plain loop in numpy scalars of the value type: products rounded to
    # the type, added in A-then-B stored order from +0.0
    A = _rand_csr(wl.seed(78), 30, 25, 7, vt)
    B = _rand_csr(wl.seed(79), 25, 35, 7, vt)
    r = oracle.spgemm(A, B)
    arp, brp = A.rowptr.astype(np.int64), B.rowptr.astype(np.int64)
    T = np.dtype(vt).type
    for i in range(A.nrows):
        acc = {}
        for p in range(arp[i], arp[i + 1]):
            j = int(A.col[p])
            for q in range(brp[j], brp[j + 1]):
                k = int(B.col[q])
                prod = T(A.val[p]) * T(B.val[q])
                acc[k] = T(acc.get(k, T(0.0)) + prod)
        cols = sorted(acc)
        got = r.val[r.rowptr[i]:r.rowptr[i + 1]]
        want = np.array([acc[k] for k in cols], dtype=vt).astype(np.float64)
        assert np.array_equal(got.view(np.int64), want.view(np.int64))


# ---------------------------------------------------------------- ideal volume, hand count
def _counted_gustavson_bytes(A, B, w):
    """Bytes a two-phase Gustavson product reads and writes when every array
    access is tallied at its own width w[name]: the symbolic phase reads A's
    row pointers, A's columns, both row pointers of every referenced B row
    and B's columns; the numeric phase reads all of those again plus A's and
    B's values, and writes C (Section 4.3: B rows are not reused)."""
    rd = 0
    arp, brp = A.rowptr.astype(np.int64), B.rowptr.astype(np.int64)
    nnz_c = 0
    for phase in ("symbolic", "numeric"):
        rd += (A.nrows + 1) * w["rp_a"]          # A.rowPtr, one pass per phase
        for i in range(A.nrows):
            seen = set()
            for p in range(arp[i], arp[i + 1]):
                rd += w["col_a"]                  # A.col[p]
                if phase == "numeric":
                    rd += w["val"]                # A.val[p]
                j = int(A.col[p])
                rd += 2 * w["rp_b"]               # B.rowPtr[j], B.rowPtr[j + 1]
                for q in range(brp[j], brp[j + 1]):
                    rd += w["col_b"]              # B.col[q]
                    if phase == "numeric":
                        rd += w["val"]            # B.val[q]
                    seen.add(int(B.col[q]))
            if phase == "numeric":
                nnz_c += len(seen)
    wr = (A.nrows + 1) * w["rp_c"] + nnz_c * (w["col_c"] + w["val"])
    return rd, wr, nnz_c


def test_ideal_volume_matches_hand_count():
    # widths that differ for every array, so a dropped term, a term with the
    # wrong width or a wrong factor changes the total
    w = dict(rp_a=2, rp_b=3, col_a=5, col_b=7, val=11, rp_c=13, col_c=17)
    D1 = np.array([[1, 0, 2], [0, 0, 0], [3, 4, 5]], dtype=np.float64)
    D2 = np.array([[0, 6, 0], [7, 0, 8], [9, 1, 0]], dtype=np.float64)
    A, B = csr_from_dense(D1), csr_from_dense(D2)
    rd, wr, nnz_c = _counted_gustavson_bytes(A, B, w)
    ipv = int(oracle.ip(A, B).sum())
    assert ipv == (1 + 2) + (1 + 2 + 2)  # row 0: B rows 0, 2; row 2: B rows 0, 1, 2
    assert nnz_c == oracle.spgemm(A, B).nnz == 5
    r, wv = oracle.ideal_volume(A.nrows, A.nnz, ipv, A.nrows, nnz_c, s_rp_a=w["rp_a"],
                                s_rp_b=w["rp_b"], s_col_a=w["col_a"], s_col_b=w["col_b"],
                                s_val=w["val"], s_rp_c=w["rp_c"], s_col_c=w["col_c"])
    assert (r, wv) == (rd, wr)
    # the same on a random rectangular case
    A = _rand_csr(wl.seed(80), 17, 13, 4, np.float64)
    B = _rand_csr(wl.seed(81), 13, 19, 5, np.float64)
    rd, wr, nnz_c = _counted_gustavson_bytes(A, B, w)
    r, wv = oracle.ideal_volume(A.nrows, A.nnz, int(oracle.ip(A, B).sum()), A.nrows, nnz_c,
                                s_rp_a=w["rp_a"], s_rp_b=w["rp_b"], s_col_a=w["col_a"],
                                s_col_b=w["col_b"], s_val=w["val"], s_rp_c=w["rp_c"],
                                s_col_c=w["col_c"])
    assert (r, wv) == (rd, wr)
