"""Products run through the checked build of the library (guard bytes
around every plan allocation, verified after each plan and numeric phase;
loaded through MAGNUS_LIB by tests/test_gpu_checked.py in a process of its
own).  Each case is compared with the oracle; prints one line per case and
"checked cases ok" at the end."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import oracle  # noqa: E402
import workloads as wl  # noqa: E402
from gpu_util import compare, gpu_product  # noqa: E402


def main():
    import torch

    import paper_2501_07056_amd as mg
    assert os.environ.get("MAGNUS_LIB", "").endswith("libmagnus_checked.so")
    ctx = mg.Context(0)
    R, _ = wl.config2(12)
    Ri = wl.CSR(R.nrows, R.ncols, R.rowptr, R.col, wl.values(R.nnz, wl.seed(130), "int", np.float64))
    E = wl.erdos_renyi(600, 800, 9, wl.seed(131), val_kind="int")
    F = wl.erdos_renyi(800, 1 << 15, 30, wl.seed(132), val_kind="int")
    cases = [
        ("rmat12 auto", Ri, Ri, {}),
        ("rmat12 runs", Ri, Ri, dict(force_category="chunked", chunk_runs=1, chunk_shift=8)),
        ("rmat12 products", Ri, Ri, dict(force_category="chunked", chunk_runs=-1, chunk_shift=8)),
        ("rmat12 coarse", Ri, Ri, dict(force_category="chunked", chunk_shift=6, coarse_chunks=4)),
        ("er sort", E, F, dict(force_category="sort")),
        ("er dense", E, F, dict(force_category="dense")),
        ("er runs", E, F, dict(force_category="chunked", chunk_runs=1, chunk_shift=10)),
    ]
    for name, A, B, opts in cases:
        rp, col, val, info = gpu_product(ctx, A, B, **opts)
        compare(rp, col, val, oracle.spgemm(A, B), np.float64, exact=True)
        ctx.set_options(force_category="auto", chunk_runs=0, chunk_shift=0, coarse_chunks=0)
        print(f"{name}: ok (nnz {info['nnz_c']})", flush=True)
    # a batch with a CHUNKED product inside, eager and through the graph
    small = [wl.erdos_renyi(n, n, 6, wl.seed(140 + n), val_kind="int", val_dtype=np.float64,
                            rowptr_dtype=np.int32, col_dtype=np.int32) for n in (300, 700, 1200)]
    pairs_host = [(X, X) for X in small] + [(Ri, Ri)]
    pairs = []
    for A, B in pairs_host:
        dA = mg.DeviceCSR.from_host(A)
        pairs.append((dA, dA))
    ctx.set_options(chunk_shift=8, sort_max=65)
    bp = ctx.batch_plan(pairs)
    for graph in (False, True):
        outs = bp.execute(graph=graph)
        torch.cuda.synchronize()
        for C, (A, B) in zip(outs, pairs_host):
            rp, col, val = C.to_host()
            compare(rp.astype(np.int64), col.astype(np.int64), val.astype(np.float64),
                    oracle.spgemm(A, B), np.float64, exact=True)
        print(f"batch graph={graph}: ok", flush=True)
    bp.destroy()
    ctx.close()
    print("checked cases ok", flush=True)


if __name__ == "__main__":
    main()
