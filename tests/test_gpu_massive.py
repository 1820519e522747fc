"""Parity on the paper's massive uniform random test set (Section 4.3,
Fig. 9), scaled to test time: 1024 rows of C, d entries per row of A and of
every referenced row of B, m_C swept past one coarse chunk, with the coarse
level and without it (the paper's ablation).  Rows drawn at random are compared with
the oracle computed for those rows alone (structure exactly, values within
rtol * sum|a_ik b_kj|, rtol 1e-5 for f32)."""
import numpy as np
import pytest

import workloads as wl

from gpu_util import log
from test_gpu_fullsize import _check_rows

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("log_mc,coarse",
                         [(18, 0), (22, 0), (27, 0), (27, -1), (28, 0), (30, 0), (31, 0)])
def test_massive_er_sampled(log_mc, coarse):
    import torch

    import paper_2501_07056_amd as mg
    A, B = wl.massive_er(log_mc, d=512, nrows=1024)
    log(f"massive er 2^{log_mc} columns, coarse_chunks={coarse}: nnz(B)={B.nnz}")
    dA, dB = mg.DeviceCSR.from_host(A), mg.DeviceCSR.from_host(B)
    ctx = mg.Context(0, coarse_chunks=coarse)
    try:
        p = ctx.plan(dA, dB)
        info = p.info.as_dict()
        C = p.execute(rowptr_dtype=torch.int64)
        torch.cuda.synchronize()
        p.destroy()
        assert info["ip_total"] == 1024 * 512 * 512
        # one coarse chunk spans 2^20 columns under the full LDS budget;
        # coarse chunks of <= 1024 products skip the fine level (2^30: about
        # 256 products each, 2^31: about 128).  The first reorder runs its
        # longest tiles at 1024 threads up to 2^28 columns, at 512 threads
        # at 2^30 (over 512 coarse chunks per row); the level-2 reorder runs
        # 1024 threads at 2^22 and 256 at 2^27 and 2^28 (coarse chunks of
        # about 2^11 and 2^10 products)
        assert (info["coarse_rows"] > 0) == (coarse == 0 and log_mc > 20)
        if log_mc in (30, 31):
            assert info["coarse_fine_chunks"] == 0
        if log_mc in (22, 27) and coarse == 0:
            assert info["coarse_fine_chunks"] > 0
        rng = np.random.default_rng(log_mc)
        rows = np.concatenate([[0, A.nrows - 1], rng.choice(A.nrows, 40, replace=False)])
        _check_rows(C, A, B, rows, np.float32)
        del C
    finally:
        ctx.close()
