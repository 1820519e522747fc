"""Parity at the full workload sizes (GPU), in the launch configuration the
benchmark times: the whole product runs on the device, then rows drawn at
random (and the heaviest rows) are compared with the oracle computed for
those rows alone.  Structure must match exactly; values within
rtol * sum|a_ik b_kj| (1e-12 for f64, 1e-5 for f32)."""
import numpy as np
import pytest

import oracle
import workloads as wl

from gpu_util import RTOL, log

pytestmark = pytest.mark.gpu


def _check_rows(C, A, B, rows, vt):
    rows = np.unique(np.asarray(rows, dtype=np.int64))
    ref = oracle.spgemm(A, B, rows)
    rp = C.rowptr.cpu().numpy().astype(np.int64)
    import torch
    idx = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows])
    it = torch.from_numpy(idx).to(C.col.device)
    col = C.col[it].cpu().numpy().astype(np.int64)
    val = C.val[it].cpu().numpy().astype(np.float64)
    assert np.array_equal(np.diff(ref.rowptr), rp[rows + 1] - rp[rows]), "row lengths differ"
    assert np.array_equal(col, ref.col), "columns differ"
    assert not np.signbit(val[val == 0]).any(), "-0.0 in C"
    err = np.abs(val - ref.ref)
    bad = err > RTOL[np.dtype(vt)] * ref.abssum
    assert not bad.any(), f"{bad.sum()} values beyond tolerance"
    # row pointers are monotone and end at nnz(C)
    assert (np.diff(rp) >= 0).all() and rp[-1] == C.col.numel()
    return len(rows), len(col)


def test_config2_rmat20_sampled():
    import torch

    import paper_2501_07056_amd as mg
    A, _ = wl.config2(20)
    log(f"config2 scale 20: nnz(A)={A.nnz}")
    dA = mg.DeviceCSR.from_host(A)
    ctx = mg.Context(0)
    try:
        p = ctx.plan(dA, dA)
        info = p.info.as_dict()
        C = p.execute(rowptr_dtype=torch.int64)
        torch.cuda.synchronize()
        p.destroy()
        assert info["ip_total"] == int(oracle.ip(A, A).sum())
        assert info["rows_by_category"][2] > 0  # CHUNKED rows present
        ip = oracle.ip(A, A)
        rng = np.random.default_rng(20)
        heavy = np.argsort(-ip)[:3]
        rows = np.concatenate([heavy, rng.choice(A.nrows, 300, replace=False)])
        nr, ne = _check_rows(C, A, A, rows, np.float64)
        log(f"checked {nr} rows, {ne} entries")
        del C
    finally:
        ctx.close()


# forced to CHUNKED, the rows span 2^24 columns and take the coarse level;
# their coarse chunks hold about 16 products each and are sorted directly,
# so no per-chunk arrays of rows x chunks are built (the default category of
# these rows is SORT)
@pytest.mark.parametrize("cat,logn", [("auto", 24), ("chunked", 22), ("chunked", 24)])
def test_config3_er_sampled(cat, logn):
    import torch

    import paper_2501_07056_amd as mg
    A, B = wl.config3(logn)
    log(f"config3 2^{logn} cat={cat}")
    dA, dB = mg.DeviceCSR.from_host(A), mg.DeviceCSR.from_host(B)
    ctx = mg.Context(0, force_category=cat)
    try:
        p = ctx.plan(dA, dB)
        info = p.info.as_dict()
        C = p.execute(rowptr_dtype=torch.int64)
        torch.cuda.synchronize()
        p.destroy()
        assert info["ip_total"] == 256 << logn  # every row: 16 entries times 16
        rng = np.random.default_rng(24)
        rows = np.concatenate([[0, A.nrows - 1], rng.choice(A.nrows, 2000, replace=False)])
        _check_rows(C, A, B, rows, np.float32)
        del C
    finally:
        ctx.close()


def test_config4_batch512_sampled():
    import torch

    import paper_2501_07056_amd as mg
    pairs_host = wl.config4()
    pairs = []
    for Ah, _ in pairs_host:
        d = mg.DeviceCSR.from_host(Ah)
        pairs.append((d, d))
    ctx = mg.Context(0)
    try:
        bp = ctx.batch_plan(pairs)
        outs = bp.execute()
        torch.cuda.synchronize()
        rng = np.random.default_rng(4)
        for b in range(0, len(pairs), 17):
            A = pairs_host[b][0]
            rows = rng.choice(A.nrows, min(100, A.nrows), replace=False)
            _check_rows(outs[b], A, A, rows, np.float32)
        bp.destroy()
    finally:
        ctx.close()
