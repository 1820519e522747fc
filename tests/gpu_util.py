"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
compare with the CPU oracle element by element."""
from __future__ import annotations

import sys

import numpy as np

import oracle

RTOL = {np.dtype(np.float64): 1e-12, np.dtype(np.float32): 1e-5}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_product(ctx, A, B, rowptr_dtype="int64", **opts):
    """C = A*B on cuda:0 from host CSR operands; returns host arrays and info."""
    import torch

    import paper_2501_07056_amd as mg
    if opts:
        ctx.set_options(**opts)
    dA = mg.DeviceCSR.from_host(A)
    dB = dA if B is A else mg.DeviceCSR.from_host(B)
    p = ctx.plan(dA, dB)
    try:
        C = p.execute(rowptr_dtype=getattr(torch, rowptr_dtype))
        torch.cuda.synchronize()
        info = p.info.as_dict()
    finally:
        p.destroy()
    rp, col, val = C.to_host()
    return rp.astype(np.int64), col.astype(np.int64), val.astype(np.float64), info


def compare(rp, col, val, ref: oracle.OracleC, vdtype, exact: bool, rows=None):
    """Structure must match exactly; values bit-exactly (exact) or within
    rtol * sum|products| of the long-double oracle sum.  No -0.0 anywhere."""
    if rows is None:
        assert np.array_equal(rp, ref.rowptr), "row pointers differ"
        assert np.array_equal(col, ref.col), "columns differ"
        got = val
    else:
        parts_c, parts_v = [], []
        for i in rows:
            parts_c.append(col[rp[i]:rp[i + 1]])
            parts_v.append(val[rp[i]:rp[i + 1]])
        gc = np.concatenate(parts_c) if parts_c else np.zeros(0, np.int64)
        got = np.concatenate(parts_v) if parts_v else np.zeros(0)
        assert np.array_equal(np.diff(ref.rowptr), np.array([rp[i + 1] - rp[i] for i in rows])), \
            "row lengths differ"
        assert np.array_equal(gc, ref.col), "columns differ"
    zeros = got == 0
    assert not np.signbit(got[zeros]).any(), "-0.0 in C"
    if exact:
        assert np.array_equal(got, ref.val), "values differ (exact)"
        return 0.0
    rtol = RTOL[np.dtype(vdtype)]
    err = np.abs(got - ref.ref)
    bound = rtol * ref.abssum
    bad = err > bound
    assert not bad.any(), f"{bad.sum()} values beyond rtol*sum|p| (max err/scale " \
                          f"{np.max(err / np.maximum(ref.abssum, 1e-300)):.3e})"
    return float(np.max(err / np.maximum(ref.abssum, 1e-300))) if len(err) else 0.0
