"""Seeded synthetic CSR inputs (shared by the GPU path's tests/bench and the
oracle's tests).  This module draws patterns and values only; it computes
nothing of the SpGEMM itself.

The workloads stand in for the paper's test sets (Section 4.2, Table 3): the
R-MAT "RMat16" matrices (Graph500 parameters a=.57, b=c=.19, 16 entries per
row), uniform random (Erdos-Renyi) matrices, and banded matrices.  The
SuiteSparse collection is not used.

Seeds: seed_k = 2501070560 + k.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.cpp")
_LIB = os.path.join(_HERE, "_gen.so")

SEED_BASE = 2501070560


def seed(k: int) -> int:
    return SEED_BASE + k


def build(force: bool = True) -> str:
    """Compile the generator library in-tree with g++."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, u64, i32, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        lib.wl_draw.argtypes = [u64, u64, u64]
        lib.wl_draw.restype = u64
        lib.wl_er.argtypes = [i64, i64, i32, u64, P, P, i32, i32]
        lib.wl_er.restype = i32
        lib.wl_er_wide.argtypes = [i64, i64, i32, u64, P, P, P, i32, i32]
        lib.wl_er_wide.restype = i64
        lib.wl_banded.argtypes = [i64, i64, i32, u64, P, P, i32, i32]
        lib.wl_banded.restype = i64
        lib.wl_rmat.argtypes = [i32, i64, dbl, dbl, dbl, u64, i32, P, P, i32, i32]
        lib.wl_rmat.restype = i64
        lib.wl_values.argtypes = [i64, u64, i32, P, i32, i32]
        lib.wl_values.restype = i32
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


@dataclass
class CSR:
    """Host CSR matrix: rowptr (int32/int64), col (int32/int64), val (f32/f64)."""
    nrows: int
    ncols: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def astype(self, rowptr=None, col=None, val=None) -> "CSR":
        return CSR(self.nrows, self.ncols,
                   self.rowptr.astype(rowptr or self.rowptr.dtype, copy=False),
                   self.col.astype(col or self.col.dtype, copy=False),
                   self.val.astype(val or self.val.dtype, copy=False), dict(self.meta))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.nrows, self.ncols), dtype=np.float64)
        for i in range(self.nrows):
            for p in range(int(self.rowptr[i]), int(self.rowptr[i + 1])):
                d[i, int(self.col[p])] += float(self.val[p])
        return d


def values(nnz: int, seed_: int, kind: str, dtype) -> np.ndarray:
    dtype = np.dtype(dtype)
    out = np.empty(nnz, dtype=dtype)
    if nnz:
        _load().wl_values(nnz, seed_, 1 if kind == "int" else 0, _ptr(out), dtype.itemsize, 0)
    return out


def _finish(n, m, rowptr64, col, val_seed, val_kind, val_dtype, rowptr_dtype, meta):
    nnz = int(rowptr64[-1])
    val = values(nnz, val_seed, val_kind, val_dtype)
    return CSR(n, m, rowptr64.astype(rowptr_dtype, copy=False), col, val, meta)


def erdos_renyi(n: int, m: int, d: int, seed_: int, *, val_kind="uniform", val_dtype=np.float64,
                rowptr_dtype=np.int64, col_dtype=np.int32) -> CSR:
    """n x m matrix with exactly d distinct uniform columns per row."""
    col_dtype = np.dtype(col_dtype)
    rowptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(n * d, dtype=col_dtype)
    rc = _load().wl_er(n, m, d, seed_, _ptr(rowptr), _ptr(col), col_dtype.itemsize, 0)
    if rc != 0:
        raise ValueError("wl_er failed")
    return _finish(n, m, rowptr, col, seed_ + 7919, val_kind, val_dtype, rowptr_dtype,
                   {"kind": "er", "d": d, "seed": seed_})


def erdos_renyi_wide(n: int, m: int, d: int, seed_: int, *, rows_mask=None, val_kind="uniform",
                     val_dtype=np.float32, rowptr_dtype=np.int64, col_dtype=np.int32) -> CSR:
    """n x m with d distinct uniform columns in each row that rows_mask names
    (every row if None), the other rows empty; for m >= 2d, fast for large d."""
    col_dtype = np.dtype(col_dtype)
    if m > np.iinfo(col_dtype).max + 1:
        raise ValueError("column type too narrow for m")
    rowptr = np.empty(n + 1, dtype=np.int64)
    if rows_mask is not None:
        rows_mask = np.ascontiguousarray(rows_mask, dtype=np.uint8)
        assert rows_mask.shape == (n,)
        nr = int(rows_mask.sum())
    else:
        nr = n
    col = np.empty(nr * d, dtype=col_dtype)
    nnz = _load().wl_er_wide(n, m, d, seed_, None if rows_mask is None else _ptr(rows_mask),
                             _ptr(rowptr), _ptr(col), col_dtype.itemsize, 0)
    if nnz < 0:
        raise ValueError("wl_er_wide failed")
    return _finish(n, m, rowptr, col, seed_ + 7919, val_kind, val_dtype, rowptr_dtype,
                   {"kind": "er_wide", "d": d, "seed": seed_})


def banded(n: int, w: int, k: int, seed_: int, *, val_kind="uniform", val_dtype=np.float64,
           rowptr_dtype=np.int64, col_dtype=np.int32) -> CSR:
    """n x n: diagonal plus k distinct uniform columns within |i-j| <= w."""
    col_dtype = np.dtype(col_dtype)
    rowptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(n * (k + 1), dtype=col_dtype)
    nnz = _load().wl_banded(n, w, k, seed_, _ptr(rowptr), _ptr(col), col_dtype.itemsize, 0)
    return _finish(n, n, rowptr, col[:nnz], seed_ + 7919, val_kind, val_dtype, rowptr_dtype,
                   {"kind": "banded", "w": w, "k": k, "seed": seed_})


def rmat(scale: int, seed_: int, *, edge_factor=16, a=0.57, b=0.19, c=0.19, val_kind="uniform",
         val_dtype=np.float64, rowptr_dtype=np.int64, col_dtype=np.int32, merge=True) -> CSR:
    """R-MAT, 2^scale vertices, edge_factor * 2^scale draws, duplicates merged
    (kept, sorted within rows, when merge is False)."""
    col_dtype = np.dtype(col_dtype)
    n = 1 << scale
    rowptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(edge_factor * n, dtype=col_dtype)
    nnz = _load().wl_rmat(scale, edge_factor, a, b, c, seed_, int(bool(merge)), _ptr(rowptr), _ptr(col),
                          col_dtype.itemsize, 0)
    if nnz < 0:
        raise ValueError("wl_rmat failed")
    col = col[:nnz].copy()
    return _finish(n, n, rowptr, col, seed_ + 7919, val_kind, val_dtype, rowptr_dtype,
                   {"kind": "rmat", "scale": scale, "seed": seed_, "draws": edge_factor * n})


def uniform01(seed_: int, stream: int, k: int) -> float:
    return (int(_load().wl_draw(seed_, stream, k)) >> 11) * (1.0 / 9007199254740992.0)


# ---------------------------------------------------------------------------
# The five workloads.  Each returns operands; smaller variants for parity
# tests take a size argument.
# ---------------------------------------------------------------------------

def config1(n: int = 4096, d: int = 8):
    """C = A*A; A is n x n Erdos-Renyi, exactly d per row, integer values in
    [-4, 4] stored as f64 (all partial sums exact), int32 indices."""
    A = erdos_renyi(n, n, d, seed(1), val_kind="int", val_dtype=np.float64,
                    rowptr_dtype=np.int32, col_dtype=np.int32)
    return A, A


def config2(scale: int = 20):
    """C = A*A; A is R-MAT (a=.57, b=c=.19, d=.05), 16 draws per row, merged,
    f64 uniform values, int32 indices (C takes int64 row pointers)."""
    A = rmat(scale, seed(2), val_kind="uniform", val_dtype=np.float64,
             rowptr_dtype=np.int32, col_dtype=np.int32)
    return A, A


def config3(logn: int = 24, d: int = 16):
    """C = A*B; A, B independent n x n Erdos-Renyi, exactly d per row, f32
    uniform values, int64 row pointers, int32 columns."""
    n = 1 << logn
    A = erdos_renyi(n, n, d, seed(3), val_kind="uniform", val_dtype=np.float32,
                    rowptr_dtype=np.int64, col_dtype=np.int32)
    B = erdos_renyi(n, n, d, seed(33), val_kind="uniform", val_dtype=np.float32,
                    rowptr_dtype=np.int64, col_dtype=np.int32)
    return A, B


def massive_er(log_mc: int, d: int = 1024, nrows: int = 4096):
    """The uniform random test set of Section 4.3 (Fig. 9): C has `nrows` rows
    and 2^log_mc columns; every row of A has d distinct uniform columns and
    every row of B that A references has d distinct uniform columns in
    [0, 2^log_mc); the rows of B that no entry of A references are empty.

    A's column space (the rows of B) is nrows * d wide instead of 2^log_mc:
    only referenced rows of B exist either way, so the product has the same
    statistics, and B's row pointers stay small.  f32 values uniform in
    [-1, 1); int64 row pointers; int32 columns up to 2^31 columns, int64
    beyond."""
    mc = 1 << log_mc
    k = nrows * d
    A = erdos_renyi_wide(nrows, k, d, seed(6), val_dtype=np.float32,
                         col_dtype=np.int32 if k <= (1 << 31) else np.int64)
    mask = np.zeros(k, dtype=np.uint8)
    mask[A.col] = 1
    B = erdos_renyi_wide(k, mc, d, seed(66), rows_mask=mask, val_dtype=np.float32,
                         col_dtype=np.int32 if mc <= (1 << 31) else np.int64)
    return A, B


def config4_shapes(count: int = 512, lo: int = 1024, hi: int = 65536, dlo: int = 4, dhi: int = 32):
    """Row counts log-uniform in [lo, hi] and d uniform in [dlo, dhi]."""
    shapes = []
    for b in range(count):
        u = uniform01(seed(4), 100, 2 * b)
        n = int(round(math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))))
        v = uniform01(seed(4), 100, 2 * b + 1)
        d = dlo + min(dhi - dlo, int(v * (dhi - dlo + 1)))
        shapes.append((n, d))
    return shapes


def config4(count: int = 512, lo: int = 1024, hi: int = 65536, dlo: int = 4, dhi: int = 32):
    """Batched: count independent C_b = A_b*A_b, A_b Erdos-Renyi, f32, int32."""
    mats = []
    for b, (n, d) in enumerate(config4_shapes(count, lo, hi, dlo, dhi)):
        A = erdos_renyi(n, n, d, seed(1000 + b), val_kind="uniform", val_dtype=np.float32,
                        rowptr_dtype=np.int32, col_dtype=np.int32)
        mats.append((A, A))
    return mats


@dataclass
class Request:
    rid: int
    arrival_s: float
    kind: str       # "rmat" or "banded"
    n: int
    a_seed: int
    b_seed: int


def config5_requests(count: int = 2000, qps: float = 10.0, lo: float = 1e3, hi: float = 1e6,
                     max_scale: int = 20):
    """Poisson request stream: exponential gaps at rate qps; n log-uniform in
    [lo, hi]; half R-MAT (scale = round(log2 n), A and B independent) and half
    banded (w=64, 8 off-diagonal entries per row).  Values are f64 uniform."""
    reqs = []
    t = 0.0
    for r in range(count):
        u_gap = uniform01(seed(5), 200, 4 * r)
        t += -math.log(1.0 - u_gap) / qps
        u_n = uniform01(seed(5), 200, 4 * r + 1)
        n = int(round(math.exp(math.log(lo) + u_n * (math.log(hi) - math.log(lo)))))
        kind = "rmat" if uniform01(seed(5), 200, 4 * r + 2) < 0.5 else "banded"
        if kind == "rmat":
            sc = min(max_scale, max(1, int(round(math.log2(n)))))
            n = 1 << sc
        reqs.append(Request(r, t, kind, n, seed(10000 + 2 * r), seed(10001 + 2 * r)))
    return reqs


def config5_operand(kind: str, n: int, seed_: int) -> CSR:
    if kind == "rmat":
        sc = int(round(math.log2(n)))
        return rmat(sc, seed_, val_kind="uniform", val_dtype=np.float64,
                    rowptr_dtype=np.int32, col_dtype=np.int32)
    return banded(n, 64, 8, seed_, val_kind="uniform", val_dtype=np.float64,
                  rowptr_dtype=np.int32, col_dtype=np.int32)
