"""Full-size parity, run by hand once on a GPU (not collected by pytest): C
of the R-MAT scale-20 square (C = A*A, f64, int32) or the Erdos-Renyi 2^24
product (C = A*B, 16 per row, f32) computed on the device, then every row
compared with the CPU oracle, block by block of rows: row lengths and
columns exactly, values within rtol * sum |a_ik b_kj| of the oracle's
long-double sum (the tests' tolerance).  Prints one line per block and a
final JSON line.

    python -u tests/full_parity.py rmat20 [--block-entries 100000000]
    python -u tests/full_parity.py er24
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import oracle  # noqa: E402
import workloads as wl  # noqa: E402
from gpu_util import RTOL  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["rmat20", "er24"])
    ap.add_argument("--block-entries", type=int, default=100_000_000)
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    import torch

    import paper_2501_07056_amd as mg
    t0 = time.time()
    A, B = wl.config2(20) if args.workload == "rmat20" else wl.config3(24)
    vt = np.dtype(A.val.dtype)
    print(f"[parity] {args.workload}: generated in {time.time() - t0:.1f} s", flush=True)
    ctx = mg.Context(0)
    dA = mg.DeviceCSR.from_host(A)
    dB = dA if B is A else mg.DeviceCSR.from_host(B)
    t0 = time.time()
    C = ctx.spgemm(dA, dB)
    torch.cuda.synchronize()
    print(f"[parity] C on the device in {time.time() - t0:.2f} s, nnz {C.col.numel()}", flush=True)
    rp = C.rowptr.cpu().numpy().astype(np.int64)
    n = A.nrows
    rtol = RTOL[vt]
    rows_done, entries, worst, bad_struct, bad_val, neg0 = 0, 0, 0.0, 0, 0, 0
    t_start = time.time()
    r0 = 0
    while r0 < n:
        # rows of about block_entries outputs
        r1 = int(np.searchsorted(rp, rp[r0] + args.block_entries, side="right")) - 1
        r1 = min(max(r1, r0 + 1), n)
        rows = np.arange(r0, r1, dtype=np.int64)
        ref = oracle.spgemm(A, B, rows, nthreads=args.threads)
        lo, hi = int(rp[r0]), int(rp[r1])
        col = C.col[lo:hi].cpu().numpy().astype(np.int64)
        val = C.val[lo:hi].cpu().numpy().astype(np.float64)
        if not (np.array_equal(np.diff(ref.rowptr), np.diff(rp[r0:r1 + 1])) and
                np.array_equal(col, ref.col)):
            bad_struct += 1
        else:
            err = np.abs(val - ref.ref)
            scale = np.maximum(ref.abssum, 1e-300)
            bad_val += int((err > rtol * ref.abssum).sum())
            if len(err):
                worst = max(worst, float((err / scale).max()))
            z = val == 0
            neg0 += int(np.signbit(val[z]).sum())
        rows_done += len(rows)
        entries += hi - lo
        del ref, col, val
        print(f"[parity] rows {r0}..{r1} ({rows_done / n:.1%}), entries {entries}, "
              f"{time.time() - t_start:.0f} s, structure blocks bad {bad_struct}, "
              f"values bad {bad_val}, max err/scale {worst:.3e}", flush=True)
        r0 = r1
    out = {"workload": args.workload, "rows": n, "entries": entries, "nnz_C": int(rp[-1]),
           "value_dtype": str(vt), "rtol": rtol, "blocks_with_structure_mismatch": bad_struct,
           "values_beyond_rtol": bad_val, "negative_zeros": neg0,
           "max_err_over_sum_abs": worst, "seconds": round(time.time() - t_start, 1),
           "all_equal_within_rtol": bad_struct == 0 and bad_val == 0 and neg0 == 0}
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
