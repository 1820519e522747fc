"""Coarse level of the method (Section 3.3, Algorithm 4) as plain sequential
loops on host CSR matrices.  Test infrastructure only.

For the rows of C listed in ``coarse_rows_c`` (the paper's coarseRowsC):

1. coarseRowsB, the rows of B the outer product needs, from a bitmap over
   the entries of the submatrix A_hat of A made of those rows;
2. A_hat in CSC form, built the usual way: a histogram of the entries per
   column, an exclusive prefix sum into the column pointers, then the row
   indices (positions in coarse_rows_c) and values placed column by column;
3. a histogram of the intermediate product per (row, coarse chunk), reading
   A_hat's columns and the B rows of coarseRowsB; the coarse chunk of a
   column k is k >> cshift;
4. an exclusive prefix sum over the rows' chunk counts, where each row's
   offsets continue from the previous row's, and the reorder: the same loops
   again, every product a * b written at its (row, chunk) slot with its
   column made local to the coarse chunk.

Step 5 of the paper (the fine level inside each coarse chunk) is
``two_level_rows``: the fine reorder of each coarse chunk (Algorithm 3, see
``reorder.py``) followed by a dense accumulator per fine chunk (Algorithm 1).
"""
from __future__ import annotations

import numpy as np

from .reorder import reorder_row


def coarse_rows_b(A, coarse_rows_c):
    """Step 1: the B rows referenced by the entries of A_hat, ascending."""
    rp = A.rowptr.astype(np.int64)
    needed = np.zeros(A.ncols, dtype=bool)
    for i in coarse_rows_c:
        for p in range(int(rp[i]), int(rp[i + 1])):
            needed[int(A.col[p])] = True
    return [j for j in range(A.ncols) if needed[j]]


def csc_of_rows(A, coarse_rows_c):
    """Step 2: A_hat (the rows coarse_rows_c of A) in CSC form: column
    pointers, row positions (index into coarse_rows_c) and values."""
    rp = A.rowptr.astype(np.int64)
    counts = [0] * A.ncols
    for i in coarse_rows_c:
        for p in range(int(rp[i]), int(rp[i + 1])):
            counts[int(A.col[p])] += 1
    colptr = [0] * (A.ncols + 1)
    for j in range(A.ncols):
        colptr[j + 1] = colptr[j] + counts[j]
    fill = list(colptr[:-1])
    rows = [0] * colptr[-1]
    vals = [0.0] * colptr[-1]
    for r, i in enumerate(coarse_rows_c):
        for p in range(int(rp[i]), int(rp[i + 1])):
            j = int(A.col[p])
            rows[fill[j]] = r
            vals[fill[j]] = A.val[p]
            fill[j] += 1
    return colptr, rows, vals


def coarse_level(A, B, coarse_rows_c, cshift: int):
    """Steps 1-4.  Returns (offsets, col_coarse, val_coarse, n_chunks):
    offsets[r * n_chunks + c] is where the products of row coarse_rows_c[r]
    in coarse chunk c start (n_rows * n_chunks + 1 entries, chained across
    rows), col_coarse the columns local to the coarse chunk, val_coarse the
    products, in the outer product's order."""
    n_chunks = (B.ncols + (1 << cshift) - 1) >> cshift
    rows_b = coarse_rows_b(A, coarse_rows_c)
    colptr, hrow, hval = csc_of_rows(A, coarse_rows_c)
    brp = B.rowptr.astype(np.int64)
    nr = len(coarse_rows_c)
    counts = [[0] * n_chunks for _ in range(nr)]
    # step 3: histogram
    for j in rows_b:
        for q in range(colptr[j], colptr[j + 1]):
            r = hrow[q]
            for p in range(int(brp[j]), int(brp[j + 1])):
                counts[r][int(B.col[p]) >> cshift] += 1
    # step 4: prefix sum chained across rows, then the reorder
    offsets = [0] * (nr * n_chunks + 1)
    for r in range(nr):
        for c in range(n_chunks):
            offsets[r * n_chunks + c + 1] = offsets[r * n_chunks + c] + counts[r][c]
    fill = list(offsets[:-1])
    total = offsets[-1]
    col_coarse = np.zeros(total, dtype=np.int64)
    val_coarse = np.zeros(total, dtype=np.float64)
    for j in rows_b:
        for q in range(colptr[j], colptr[j + 1]):
            r, a = hrow[q], float(hval[q])
            for p in range(int(brp[j]), int(brp[j + 1])):
                k = int(B.col[p])
                c = k >> cshift
                slot = fill[r * n_chunks + c]
                col_coarse[slot] = k - (c << cshift)
                val_coarse[slot] = a * float(B.val[p])
                fill[r * n_chunks + c] += 1
    return np.asarray(offsets, dtype=np.int64), col_coarse, val_coarse, n_chunks


def two_level_rows(A, B, coarse_rows_c, cshift: int, shift: int):
    """Steps 1-5: each coarse chunk reordered into fine chunks of 2^shift
    columns, each fine chunk summed in a dense accumulator (slots start at
    +0.0, the bitmap keeps every touched column).  Returns one (columns,
    values) pair per row of coarse_rows_c, columns ascending."""
    offsets, colc, valc, n_chunks = coarse_level(A, B, coarse_rows_c, cshift)
    n_fine = 1 << (cshift - shift)
    out = []
    for r in range(len(coarse_rows_c)):
        cols, vals = [], []
        for c in range(n_chunks):
            s0, s1 = int(offsets[r * n_chunks + c]), int(offsets[r * n_chunks + c + 1])
            if s1 == s0:
                continue
            foff, fcol, fval = reorder_row(colc[s0:s1], valc[s0:s1], shift, 0, n_fine)
            for f in range(n_fine):
                acc = [0.0] * (1 << shift)
                seen = [False] * (1 << shift)
                for q in range(int(foff[f]), int(foff[f + 1])):
                    lc = int(fcol[q])
                    acc[lc] = acc[lc] + float(fval[q])
                    seen[lc] = True
                base = (c << cshift) + (f << shift)
                for lc in range(1 << shift):
                    if seen[lc]:
                        cols.append(base + lc)
                        vals.append(acc[lc])
        out.append((np.asarray(cols, dtype=np.int64), np.asarray(vals, dtype=np.float64)))
    return out
