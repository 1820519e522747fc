"""The serving loop (GPU): requests over registered operands are admitted by
their memory bound, batched and overlapped; every result equals the oracle
and the same product computed alone, whatever else ran beside it."""
import time

import numpy as np
import pytest

import oracle
import workloads as wl

from gpu_util import compare, log

pytestmark = pytest.mark.gpu


def _wait(srv, rids, timeout=60.0):
    t0 = time.time()
    pending = set(rids)
    while pending:
        pending = {r for r in pending if not srv.ready(r)}
        if time.time() - t0 >= timeout:
            log(f"stats at timeout: {srv.stats()}")
            for r in sorted(pending)[:8]:
                log(f"request {r}: {srv.query(r)}")
            raise AssertionError(f"requests {sorted(pending)[:5]} not finished")
        time.sleep(0.001)


def _host(C):
    rp, col, val = C.to_host()
    return rp.astype(np.int64), col.astype(np.int64), val.astype(np.float64)


def _operands(kind_vals="int"):
    """Mixed sizes: small R-MAT and banded operands (square, f64, int32)."""
    ops = []
    for sc in (8, 10, 11):
        ops.append(wl.rmat(sc, wl.seed(300 + sc), val_kind=kind_vals, val_dtype=np.float64,
                           rowptr_dtype=np.int32, col_dtype=np.int32))
    for n in (700, 3000):
        ops.append(wl.banded(n, 64, 8, wl.seed(400 + n), val_kind=kind_vals, val_dtype=np.float64,
                             rowptr_dtype=np.int32, col_dtype=np.int32))
    return ops


def test_serving_same_alone_and_in_the_mix():
    """Integer values (exact sums): each served result is bit-identical to
    the oracle and to the product computed alone through the single calls."""
    import torch

    import paper_2501_07056_amd as mg
    ops = _operands("int")
    dev = [mg.DeviceCSR.from_host(X) for X in ops]
    srv = mg.Server(0, max_batch=4, streams=2)
    ctx = mg.Context(0)
    try:
        ids = [srv.register(X) for X in dev]
        pairs = [(i, i) for i in range(len(ops))] + [(0, 0), (2, 2), (4, 4), (3, 3)]
        log(f"serving {len(pairs)} requests")
        rids = [srv.submit(a, b) for a, b in pairs]
        _wait(srv, rids)
        st = srv.stats()
        assert st["completed"] == len(rids) and st["failed"] == 0 and st["rejected"] == 0, st
        for rid, (a, b) in zip(rids, pairs):
            info = srv.query(rid)
            assert info["state"] == "done" and info["latency_ms"] >= info["queue_ms"] >= 0
            C = srv.result(rid)
            torch.cuda.synchronize()
            got = _host(C)
            ref = oracle.spgemm(ops[a], ops[b])
            compare(*got, ref, np.float64, exact=True)
            assert info["nnz"] == ref.nnz
            alone = ctx.spgemm(dev[a], dev[b])
            torch.cuda.synchronize()
            for x, y in zip(got, _host(alone)):
                assert np.array_equal(x, y), f"request {rid}: served != alone"
            srv.release(rid)
        assert srv.stats()["reserved_bytes"] == 0
    finally:
        srv.close()
        ctx.close()


def test_serving_small_budget_queues_and_random_values():
    """A budget that holds only a few requests at once: requests wait for
    memory, are admitted as earlier ones are released, and all finish within
    the f64 tolerance."""
    import torch

    import paper_2501_07056_amd as mg
    ops = _operands("uniform")
    dev = [mg.DeviceCSR.from_host(X) for X in ops]
    ctx = mg.Context(0)
    ip, nb = ctx.batch_bound([(d, d) for d in dev])
    ctx.close()
    # room for about two of the largest request's bounds
    big = max(nb) * 12 + 3001 * 8
    srv = mg.Server(0, memory_budget_bytes=int(2.5 * big + (64 << 20)), max_batch=3, streams=2,
                    workspace_cap_bytes=16 << 20)
    try:
        ids = [srv.register(X) for X in dev]
        pairs = [(i % len(ops), i % len(ops)) for i in range(20)]
        rids = [srv.submit(a, b) for a, b in pairs]
        done = set()
        t0 = time.time()
        peak = 0
        while len(done) < len(rids):
            st = srv.stats()
            peak = max(peak, st["reserved_bytes"])
            for rid, (a, b) in zip(rids, pairs):
                if rid in done or not srv.ready(rid):
                    continue
                C = srv.result(rid)
                torch.cuda.synchronize()
                compare(*_host(C), oracle.spgemm(ops[a], ops[b]), np.float64, exact=False)
                srv.release(rid)
                done.add(rid)
            assert time.time() - t0 < 120
            time.sleep(0.001)
        st = srv.stats()
        assert st["completed"] == 20 and st["failed"] == 0, st
        assert peak <= st["budget_bytes"], (peak, st)
        assert st["peak_reserved_bytes"] <= st["budget_bytes"], st
        assert st["reserved_bytes"] == 0, st
    finally:
        srv.close()


def test_serving_exact_probe_and_rejection():
    """A request whose bound exceeds the budget but whose exact size fits is
    planned exactly and served; one whose exact size does not fit is
    rejected."""
    import paper_2501_07056_amd as mg
    # every A row picks 8 of 16 B rows; all B rows hold the same 1000
    # columns: ip = 8000 per row, nnz(C) = 1000 per row
    n, k, m = 400, 16, 100000
    rng = np.random.default_rng(5)
    arp = np.arange(0, 8 * n + 1, 8, dtype=np.int32)
    acol = np.concatenate([np.sort(rng.choice(k, 8, replace=False)) for _ in range(n)]).astype(np.int32)
    A = wl.CSR(n, k, arp, acol, rng.integers(-3, 4, size=8 * n).astype(np.float64))
    cols = np.sort(rng.choice(m, 1000, replace=False)).astype(np.int32)
    B = wl.CSR(k, m, np.arange(0, 1000 * k + 1, 1000, dtype=np.int32), np.tile(cols, k),
               rng.integers(-3, 4, size=1000 * k).astype(np.float64))
    dA, dB = mg.DeviceCSR.from_host(A), mg.DeviceCSR.from_host(B)
    exact_c = 1000 * n * 12 + (n + 1) * 8
    bound_c = 8000 * n * 12
    srv = mg.Server(0, memory_budget_bytes=int(exact_c * 1.5 + (8 << 20)),
                    workspace_cap_bytes=1 << 20)
    try:
        assert srv.stats()["budget_bytes"] < bound_c
        a, b = srv.register(dA), srv.register(dB)
        rid = srv.submit(a, b)
        _wait(srv, [rid])
        assert srv.query(rid)["state"] == "done", srv.query(rid)
        st = srv.stats()
        assert st["exact_probes"] == 1 and st["peak_reserved_bytes"] <= st["budget_bytes"], st
        import torch
        C = srv.result(rid)
        torch.cuda.synchronize()
        compare(*_host(C), oracle.spgemm(A, B), np.float64, exact=True)
        srv.release(rid)
    finally:
        srv.close()
    srv = mg.Server(0, memory_budget_bytes=exact_c // 2, workspace_cap_bytes=1 << 20)
    try:
        a, b = srv.register(dA), srv.register(dB)
        rid = srv.submit(a, b)
        _wait(srv, [rid])
        assert srv.query(rid)["state"] == "rejected"
        with pytest.raises(mg.MagnusError, match="REJECTED"):
            srv.result(rid)
        srv.release(rid)
        assert srv.stats()["rejected"] == 1
    finally:
        srv.close()


@pytest.mark.parametrize("est_pct", [100, 1])
def test_serving_tight_budget_with_chunked_requests(est_pct):
    """Integer values: requests with CHUNKED rows (wide R-MAT rows) under a
    budget that holds about one of them planned: groups whose planning does
    not fit are put back and retried (forced with planning estimates at 1 %
    of the default), every request finishes with the oracle's result, and
    the reserved memory never exceeds the budget."""
    import torch

    import paper_2501_07056_amd as mg
    ops = [wl.rmat(sc, wl.seed(310 + sc), val_kind="int", val_dtype=np.float64,
                   rowptr_dtype=np.int32, col_dtype=np.int32) for sc in (13, 14)]
    ops.append(wl.banded(5000, 64, 8, wl.seed(410), val_kind="int", val_dtype=np.float64,
                         rowptr_dtype=np.int32, col_dtype=np.int32))
    dev = [mg.DeviceCSR.from_host(X) for X in ops]
    cap = 1 << 20
    # the most one request needs alone: its exact plan and C
    ctx = mg.Context(0, max_workspace_bytes=cap)
    need = []
    for d in dev:
        p = ctx.plan(d, d)
        need.append(p.info.as_dict()["plan_bytes"] + p.nnz * 12 + (d.nrows + 1) * 8)
        p.destroy()
    ctx.close()
    srv = mg.Server(0, memory_budget_bytes=int(1.3 * max(need)), workspace_cap_bytes=cap,
                    max_batch=4, streams=2, plan_estimate_pct=est_pct)
    try:
        ids = [srv.register(X) for X in dev]
        pairs = [(i % 3, i % 3) for i in range(12)]
        log(f"tight budget {srv.stats()['budget_bytes']} for {len(pairs)} requests")
        refs = {i: oracle.spgemm(ops[i], ops[i]) for i in range(3)}
        rids = [srv.submit(ids[a], ids[b]) for a, b in pairs]
        # results hold their memory until released: check and release each
        # one as it finishes, as a client would
        done, t0 = set(), time.time()
        while len(done) < len(rids):
            for rid, (a, b) in zip(rids, pairs):
                if rid in done or not srv.ready(rid):
                    continue
                info = srv.query(rid)
                assert info["state"] == "done", info
                C = srv.result(rid)
                torch.cuda.synchronize()
                compare(*_host(C), refs[a], np.float64, exact=True)
                srv.release(rid)
                done.add(rid)
            if time.time() - t0 > 60:
                log(f"stats at timeout: {srv.stats()}")
                raise AssertionError(f"{len(rids) - len(done)} requests not finished")
            time.sleep(0.001)
        st = srv.stats()
        log(f"tight budget stats {st}")
        assert st["completed"] == 12 and st["failed"] == 0 and st["rejected"] == 0, st
        assert st["peak_reserved_bytes"] <= st["budget_bytes"], st
        assert st["reserved_bytes"] == 0, st
        if est_pct == 1:
            assert st["deferred"] > 0, st
    finally:
        srv.close()


def test_serving_errors():
    import paper_2501_07056_amd as mg
    X = wl.erdos_renyi(50, 70, 3, wl.seed(7), val_dtype=np.float64)
    Y = wl.erdos_renyi(50, 50, 3, wl.seed(8), val_dtype=np.float32)
    srv = mg.Server(0)
    try:
        x = srv.register(mg.DeviceCSR.from_host(X))
        with pytest.raises(mg.MagnusError, match="DTYPE"):
            srv.register(mg.DeviceCSR.from_host(Y))
        with pytest.raises(mg.MagnusError, match="SHAPE"):
            srv.submit(x, x)  # 50x70 times 50x70
        with pytest.raises(mg.MagnusError, match="INVALID_ARG"):
            srv.submit(x, 5)
        with pytest.raises(mg.MagnusError, match="INVALID_ARG"):
            srv.release(12345)
    finally:
        srv.close()


def test_serving_arrivals_during_a_running_group_and_poll():
    """Random f64 values: requests submitted while an earlier group is still
    on the device are admitted and overlapped; each result equals the same
    product computed alone within N5 (rtol * sum|a_ik b_kj| from the oracle),
    and magnus_server_poll reports every request exactly once."""
    import torch

    import paper_2501_07056_amd as mg
    ops = _operands("uniform")
    ops.append(wl.rmat(15, wl.seed(315), val_kind="uniform", val_dtype=np.float64,
                       rowptr_dtype=np.int32, col_dtype=np.int32))
    big = len(ops) - 1
    dev = [mg.DeviceCSR.from_host(X) for X in ops]
    srv = mg.Server(0, max_batch=3, streams=2)
    ctx = mg.Context(0)
    try:
        for X in dev:
            srv.register(X)
        first = srv.submit(big, big)
        t0 = time.time()
        while srv.query(first)["state"] == "queued":
            assert time.time() - t0 < 60
            time.sleep(0.0002)
        during = srv.query(first)["state"] == "running"
        pairs = [(big, big)] + [(i % big, i % big) for i in range(12)]
        rids = [first]
        for a, b in pairs[1:]:
            rids.append(srv.submit(a, b))
            time.sleep(0.0005)
        log(f"arrivals while the first group runs: {during}")
        seen = {}
        t0 = time.time()
        while len(seen) < len(rids):
            for c in srv.poll(8):
                assert c["request_id"] not in seen, "request reported twice"
                seen[c["request_id"]] = c
            assert time.time() - t0 < 120, f"{len(seen)} of {len(rids)} reported"
            time.sleep(0.001)
        assert srv.poll(8) == []
        for rid, (a, b) in zip(rids, pairs):
            c = seen[rid]
            info = srv.query(rid)
            assert c["state"] == "done" and c["status"] == 0 and c["nnz"] == info["nnz"]
            assert abs(c["latency_ms"] - info["latency_ms"]) < 1e-6
            got = _host(srv.result(rid))
            torch.cuda.synchronize()
            alone = _host(ctx.spgemm(dev[a], dev[b]))
            torch.cuda.synchronize()
            ref = oracle.spgemm(ops[a], ops[b])
            compare(*got, ref, np.float64, exact=False)
            assert np.array_equal(got[0], alone[0]) and np.array_equal(got[1], alone[1])
            assert (np.abs(got[2] - alone[2]) <= 2e-12 * ref.abssum).all(), \
                f"request {rid}: served and alone differ beyond the tolerance"
            srv.release(rid)
        st = srv.stats()
        assert st["completed"] == len(rids) and st["failed"] == 0 and st["reserved_bytes"] == 0
    finally:
        srv.close()
        ctx.close()
