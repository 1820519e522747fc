"""Batches of products through magnus_batch_plan / magnus_batch_execute (GPU):
every product of a batch matches the CPU oracle (structure exactly, values
bit-exactly on integer data, else within rtol * sum|a_ik b_kj|), matches the
same product computed alone, and graph replays match the eager launches."""
import numpy as np
import pytest

import oracle
import workloads as wl

from gpu_util import compare, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2501_07056_amd as mg
    c = mg.Context(0)
    yield c
    c.close()


def _dev(pairs_host):
    import paper_2501_07056_amd as mg
    out = []
    for A, B in pairs_host:
        dA = mg.DeviceCSR.from_host(A)
        dB = dA if B is A else mg.DeviceCSR.from_host(B)
        out.append((dA, dB))
    return out


def _host(C):
    rp, col, val = C.to_host()
    return rp.astype(np.int64), col.astype(np.int64), val.astype(np.float64)


def _check_all(outs, pairs_host, vt, exact):
    for b, (C, (A, B)) in enumerate(zip(outs, pairs_host)):
        rp, col, val = _host(C)
        try:
            compare(rp, col, val, oracle.spgemm(A, B), vt, exact=exact)
        except AssertionError as e:
            raise AssertionError(f"product {b} (n={A.nrows}): {e}") from None


def _small_config4(count, lo=64, hi=2048, dlo=4, dhi=32, kind="uniform", vt=np.float32):
    mats = []
    for b, (n, d) in enumerate(wl.config4_shapes(count, lo, hi, dlo, dhi)):
        A = wl.erdos_renyi(n, n, d, wl.seed(1000 + b), val_kind=kind, val_dtype=vt,
                           rowptr_dtype=np.int32, col_dtype=np.int32)
        mats.append((A, A))
    return mats


def test_batch_matches_oracle_f32(ctx):
    import torch
    pairs_host = _small_config4(24)
    log(f"batch f32 count={len(pairs_host)}")
    pairs = _dev(pairs_host)
    bp = ctx.batch_plan(pairs)
    try:
        assert bp.nnz == [oracle.spgemm(A, B).nnz for A, B in pairs_host]
        outs = bp.execute()
        torch.cuda.synchronize()
        _check_all(outs, pairs_host, np.float32, exact=False)
        info = bp.info.as_dict()
        assert info["ip_total"] == sum(int(oracle.ip(A, B).sum()) for A, B in pairs_host)
        assert info["nnz_c"] == sum(bp.nnz)
    finally:
        bp.destroy()


def test_batch_integer_values_bit_exact_and_alone(ctx):
    """Integer-valued f64 (exact sums): the batch, each product alone and the
    oracle agree bit for bit, SORT and DENSE rows both present."""
    import torch
    pairs_host = _small_config4(16, lo=64, hi=4096, kind="int", vt=np.float64)
    pairs = _dev(pairs_host)
    # products alternate between the default threshold and all-DENSE rows
    sm = [1025 if b % 2 == 0 else 1 for b in range(len(pairs))]
    bp = ctx.batch_plan(pairs, sort_max=sm)
    try:
        cats = bp.info.as_dict()["rows_by_category"]
        assert cats[0] > 0 and cats[1] > 0, cats
        outs = bp.execute()
        torch.cuda.synchronize()
        _check_all(outs, pairs_host, np.float64, exact=True)
        for b, (dA, dB) in enumerate(pairs):
            ctx.set_options(sort_max=sm[b])
            alone = ctx.spgemm(dA, dB)
            torch.cuda.synchronize()
            for x, y in zip(_host(alone), _host(outs[b])):
                assert np.array_equal(x, y), f"product {b}: alone != in batch"
    finally:
        ctx.set_options(sort_max=0)
        bp.destroy()


def test_graph_replays_and_new_buffers(ctx):
    """The captured graph is replayed on new output buffers each time, with
    eager work and synchronisation in between; every replay equals the eager
    launches."""
    import torch
    pairs_host = _small_config4(12, kind="int", vt=np.float64)
    pairs = _dev(pairs_host)
    bp = ctx.batch_plan(pairs)
    try:
        eager = [_host(C) for C in bp.execute(graph=False)]
        torch.cuda.synchronize()
        for rep in range(3):
            log(f"graph replay {rep}")
            outs = bp.alloc_outputs(rowptr_dtype=torch.int32 if rep == 1 else torch.int64)
            for C in outs:
                C.col.fill_(-7)
                C.val.fill_(123.0)
            torch.cuda.synchronize()
            outs = bp.execute(outs, graph=True)
            torch.cuda.synchronize()
            scratch = torch.ones(1 << 20, device="cuda:0").sum()  # unrelated eager work
            torch.cuda.synchronize()
            del scratch
            for b, C in enumerate(outs):
                for x, y in zip(_host(C), eager[b]):
                    assert np.array_equal(x, y), f"replay {rep} product {b} differs"
        _check_all([o for o in outs], pairs_host, np.float64, exact=True)
    finally:
        bp.destroy()


def test_batch_with_chunked_products(ctx):
    """Products that have CHUNKED rows (a short chunk length forces them) are
    planned alone inside the batch; the rest stay batched."""
    import torch
    big, _ = wl.config2(11)
    small = _small_config4(6, lo=64, hi=512, vt=np.float64)
    pairs_host = small[:3] + [(big, big)] + small[3:]
    pairs = _dev(pairs_host)
    ctx.set_options(chunk_shift=8, sort_max=65)
    try:
        bp = ctx.batch_plan(pairs)
        try:
            outs = bp.execute()
            torch.cuda.synchronize()
            _check_all(outs, pairs_host, np.float64, exact=False)
            # and again through the graph with fresh buffers
            outs = bp.execute()
            torch.cuda.synchronize()
            _check_all(outs, pairs_host, np.float64, exact=False)
        finally:
            bp.destroy()
    finally:
        ctx.set_options(chunk_shift=0, sort_max=0)


def test_batch_edge_cases(ctx):
    """Products without rows, without entries, with empty B rows, and a batch
    of one."""
    import torch
    Z = wl.CSR(0, 5, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float64))
    E = wl.CSR(7, 7, np.zeros(8, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float64))
    A = wl.erdos_renyi(300, 300, 6, wl.seed(91), val_kind="int", val_dtype=np.float64,
                       rowptr_dtype=np.int32, col_dtype=np.int32)
    B5 = wl.erdos_renyi(5, 9, 2, wl.seed(92), val_kind="int", val_dtype=np.float64,
                        rowptr_dtype=np.int32, col_dtype=np.int32)
    half = wl.CSR(300, 300, np.concatenate([A.rowptr[:151], np.full(150, A.rowptr[150], np.int32)]),
                  A.col[:A.rowptr[150]].copy(), A.val[:A.rowptr[150]].copy())
    for pairs_host in ([(Z, B5), (A, A), (E, E), (A, half)], [(A, A)], [(Z, B5)]):
        log(f"edge batch of {len(pairs_host)}")
        pairs = _dev(pairs_host)
        bp = ctx.batch_plan(pairs)
        try:
            for graph in (False, True):
                outs = bp.execute(graph=graph)
                torch.cuda.synchronize()
                _check_all(outs, pairs_host, np.float64, exact=True)
        finally:
            bp.destroy()


def test_batch_errors(ctx):
    import torch

    import paper_2501_07056_amd as mg
    A32 = wl.erdos_renyi(100, 100, 4, wl.seed(93), val_dtype=np.float32)
    A64 = wl.erdos_renyi(100, 100, 4, wl.seed(94), val_dtype=np.float64)
    p32, p64 = _dev([(A32, A32), (A64, A64)])
    with pytest.raises(mg.MagnusError, match="DTYPE"):
        ctx.batch_plan([p32, p64])
    bad = wl.erdos_renyi(100, 50, 4, wl.seed(95), val_dtype=np.float32)
    (pb,) = _dev([(bad, bad)])
    with pytest.raises(mg.MagnusError, match="SHAPE"):
        ctx.batch_plan([p32, pb])
    with pytest.raises(mg.MagnusError, match="INVALID_ARG"):
        ctx.batch_plan([p32], sort_max=[0])
    bp = ctx.batch_plan([p32, p32])
    try:
        outs = bp.alloc_outputs()
        short = mg.DeviceCSR(outs[1].nrows, outs[1].ncols, outs[1].rowptr, outs[1].col[:-1],
                             outs[1].val[:-1])
        with pytest.raises(mg.MagnusError, match="CAPACITY"):
            bp.execute([outs[0], short])
        outs = bp.execute(outs)
        torch.cuda.synchronize()
        _check_all(outs, [(A32, A32), (A32, A32)], np.float32, exact=False)
    finally:
        bp.destroy()


def test_batch_chunked_products_in_the_graph(ctx):
    """Integer values: a batch whose CHUNKED products (wide R-MAT rows, both
    reorders) run inside the captured graph, on its branches, beside the SORT
    and DENSE stages.  Replays on the same buffers, then on new ones (the
    graph is captured again), each equal to the eager launches bit for bit
    and to the oracle."""
    import torch
    R, _ = wl.config2(11)
    Ri = wl.CSR(R.nrows, R.ncols, R.rowptr, R.col, wl.values(R.nnz, wl.seed(96), "int", np.float64))
    small = _small_config4(6, lo=64, hi=512, kind="int", vt=np.float64)
    pairs_host = small[:2] + [(Ri, Ri)] + small[2:4] + [(Ri, Ri)] + small[4:]
    pairs = _dev(pairs_host)
    for runs in (1, -1):
        ctx.set_options(chunk_shift=8, sort_max=65, chunk_runs=runs)
        try:
            bp = ctx.batch_plan(pairs)
            try:
                eager = [_host(C) for C in bp.execute(graph=False)]
                torch.cuda.synchronize()
                _check_all_host(eager, pairs_host, exact=True)
                outs = bp.alloc_outputs()
                for rep in range(4):
                    if rep == 2:
                        outs = bp.alloc_outputs()  # new buffers: captured again
                    log(f"chunked in graph runs={runs} replay {rep}")
                    for C in outs:
                        C.val.fill_(123.0)
                    torch.cuda.synchronize()
                    bp.execute(outs, graph=True)
                    torch.cuda.synchronize()
                    for b, C in enumerate(outs):
                        for x, y in zip(_host(C), eager[b]):
                            assert np.array_equal(x, y), f"replay {rep} product {b} differs"
            finally:
                bp.destroy()
        finally:
            ctx.set_options(chunk_shift=0, sort_max=0, chunk_runs=0)


def _check_all_host(hosts, pairs_host, exact):
    for (rp, col, val), (A, B) in zip(hosts, pairs_host):
        compare(rp, col, val, oracle.spgemm(A, B), np.float64, exact=exact)


def test_persistent_stages_match_plain_grids(ctx):
    """Integer values: each stage as one persistent kernel pulling row tiles
    from a device counter (eager and graph, the counters cleared by a kernel on
    every replay) gives the plain grids' results bit for bit.  A small batch
    is checked against the oracle; a large one (far more SORT tiles than
    resident waves, so every wave takes several runs of tiles) against the
    plain grids only."""
    import torch
    small = _small_config4(10, lo=64, hi=4096, kind="int", vt=np.float64)
    big = []
    for b in range(6):
        A = wl.erdos_renyi(120000, 120000, 5, wl.seed(1100 + b), val_kind="int",
                           val_dtype=np.float64, rowptr_dtype=np.int32, col_dtype=np.int32)
        big.append((A, A))
    for name, pairs_host in (("small", small), ("large", big)):
        pairs = _dev(pairs_host)
        sm = [1025 if b % 3 else 1 for b in range(len(pairs))]  # every third all-DENSE
        bp = ctx.batch_plan(pairs, sort_max=sm)
        try:
            plain = [_host(C) for C in bp.execute(graph=False)]
            torch.cuda.synchronize()
            if name == "small":
                _check_all_host(plain, pairs_host, exact=True)
            outs = bp.alloc_outputs()
            for rep, (graph, pers) in enumerate(((False, True), (True, True), (True, True),
                                                  (True, False), (True, True))):
                log(f"persistent {name} rep {rep} graph={graph} persistent={pers}")
                for C in outs:
                    C.val.fill_(123.0)
                torch.cuda.synchronize()
                bp.execute(outs, graph=graph, persistent=pers)
                torch.cuda.synchronize()
                for b, C in enumerate(outs):
                    for x, y in zip(_host(C), plain[b]):
                        assert np.array_equal(x, y), f"{name} rep {rep} product {b} differs"
        finally:
            bp.destroy()
