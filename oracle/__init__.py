"""CPU ORACLE -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  It shares no code with the GPU path and never
imports it.

* ``spgemm``      -- Gustavson's row-wise product (Section 2.1, Eq. 1) with an
                     ordered-map accumulator, in C++ (``oracle.cpp``).
* ``ip``          -- intermediate-product count per row (Section 4.3,
                     n_interProd).
* ``chunk_model`` -- the chunk-count model, Eqs. 2-7 of Section 3.5, as printed.
* ``reorder``     -- the fine-level histogram / prefix-sum / reorder steps of
                     Section 3.2 (Algorithm 3) on one row's products.
* ``coarse``      -- the coarse level of Section 3.3 (Algorithm 4): coarseRowsB,
                     the CSC form of the coarse rows, the outer-product
                     histogram and reorder into coarse chunks, and the fine
                     level inside each coarse chunk.
* ``ideal_volume``-- the ideal data volume of Section 4.3 (read and write
                     volumes, Eqs. 8-9).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from .chunk_model import (paper_fine_nchunks, paper_mcmax, paper_model, pow2_floor,  # noqa: F401
                          pow2_nearest, pow2_ceil)
from .volume import ideal_volume  # noqa: F401
from .reorder import reorder_row  # noqa: F401
from . import coarse  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle in-tree (g++, no contraction of multiply-add)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-shared", "-fPIC",
                               "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.oracle_ip.argtypes = [i64, i64, P, i32, P, i32, i64, i64, P, i32, P, i32, P, i64, P]
        lib.oracle_ip.restype = i64
        lib.oracle_spgemm.argtypes = [i64, i64, P, i32, P, i32, P, i64, i64, P, i32, P, i32, P,
                                      i32, P, i64, i32]
        lib.oracle_spgemm.restype = P
        lib.oracle_nnz.argtypes = [P]
        lib.oracle_nnz.restype = i64
        lib.oracle_nrows.argtypes = [P]
        lib.oracle_nrows.restype = i64
        lib.oracle_fetch.argtypes = [P, P, P, P, P, P]
        lib.oracle_fetch.restype = None
        lib.oracle_free.argtypes = [P]
        lib.oracle_free.restype = None
        _lib = lib
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _w(a):
    return int(np.asarray(a).dtype.itemsize)


@dataclass
class OracleC:
    """Rows of C for the requested rows: rowptr over those rows, col ascending,
    val (input precision, stored order), ref (long double sum), abssum."""
    rows: np.ndarray
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    ref: np.ndarray
    abssum: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


def _check(A, B):
    if A.ncols != B.nrows:
        raise ValueError("shape mismatch: A.ncols != B.nrows")
    if A.val.dtype != B.val.dtype or A.val.dtype not in (np.float32, np.float64):
        raise ValueError("values must be both float32 or both float64")


def ip(A, B, rows=None) -> np.ndarray:
    """Intermediate-product count of each requested row."""
    lib = _load()
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    cnt = A.nrows if rows_a is None else len(rows_a)
    out = np.zeros(cnt, dtype=np.int64)
    lib.oracle_ip(A.nrows, A.ncols, _p(A.rowptr), _w(A.rowptr), _p(A.col), _w(A.col),
                  B.nrows, B.ncols, _p(B.rowptr), _w(B.rowptr), _p(B.col), _w(B.col),
                  _p(rows_a), 0 if rows_a is None else len(rows_a), _p(out))
    return out


def spgemm(A, B, rows=None, nthreads: int = 0) -> OracleC:
    """Oracle product rows (all rows when ``rows`` is None)."""
    _check(A, B)
    lib = _load()
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    h = lib.oracle_spgemm(A.nrows, A.ncols, _p(A.rowptr), _w(A.rowptr), _p(A.col), _w(A.col),
                          _p(A.val), B.nrows, B.ncols, _p(B.rowptr), _w(B.rowptr), _p(B.col),
                          _w(B.col), _p(B.val), _w(A.val), _p(rows_a),
                          0 if rows_a is None else len(rows_a), int(nthreads))
    if not h:
        raise ValueError("oracle_spgemm rejected its arguments")
    try:
        nnz = lib.oracle_nnz(h)
        nr = lib.oracle_nrows(h)
        rowptr = np.zeros(nr + 1, dtype=np.int64)
        col = np.zeros(nnz, dtype=np.int64)
        val = np.zeros(nnz, dtype=np.float64)
        ref = np.zeros(nnz, dtype=np.float64)
        ab = np.zeros(nnz, dtype=np.float64)
        lib.oracle_fetch(h, _p(rowptr), _p(col), _p(val), _p(ref), _p(ab))
    finally:
        lib.oracle_free(h)
    r = np.arange(A.nrows, dtype=np.int64) if rows_a is None else rows_a
    return OracleC(r, rowptr, col, val, ref, ab)
