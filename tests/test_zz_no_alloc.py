"""The allocation-free prefix sum (GPU): magnus_exclusive_scan_i64_noalloc,
called through the C ABI, against magnus_exclusive_scan_i64 on the same
input, on two calls in a row (the second smaller, so stale partial sums of
the first would show), while the library's allocator is never asked for
memory; and a request beyond its fixed scratch is refused with nothing
launched."""
import ctypes

import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_scan_matches_the_allocating_scan():
    import torch

    import paper_2501_07056_amd as mg
    calls = {"n": 0}

    def count(nbytes):
        calls["n"] += 1
        return True

    ctx = mg.Context(0, alloc_filter=count)
    lib = ctx.lib
    try:
        g = torch.Generator(device="cpu").manual_seed(2501)
        for n in (5_000_003, 70_001):
            x = torch.randint(-(1 << 40), 1 << 40, (n,), generator=g, dtype=torch.int64).cuda()
            ref, ref_total = ctx.exclusive_scan(x)
            torch.cuda.synchronize()
            before = calls["n"]
            out = torch.full_like(x, -7)
            tot = torch.full((1,), -7, dtype=torch.int64, device="cuda")
            s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
            rc = lib.magnus_exclusive_scan_i64_noalloc(ctx.handle, ctypes.c_void_p(x.data_ptr()),
                                                       ctypes.c_void_p(out.data_ptr()), n,
                                                       ctypes.c_void_p(tot.data_ptr()), s)
            assert rc == 0, mg.MagnusError(rc, "noalloc scan")
            torch.cuda.synchronize()
            assert calls["n"] == before, "the allocation-free scan asked the allocator"
            assert torch.equal(out, ref), f"n={n}: prefix sums differ"
            assert int(tot.item()) == ref_total
            # in place, no total
            y = x.clone()
            rc = lib.magnus_exclusive_scan_i64_noalloc(ctx.handle, ctypes.c_void_p(y.data_ptr()),
                                                       ctypes.c_void_p(y.data_ptr()), n, None, s)
            assert rc == 0
            torch.cuda.synchronize()
            assert torch.equal(y, ref)
        # beyond the fixed scratch: refused before any launch (pointers unused)
        x = torch.zeros(1, dtype=torch.int64, device="cuda")
        rc = lib.magnus_exclusive_scan_i64_noalloc(ctx.handle, ctypes.c_void_p(x.data_ptr()),
                                                   ctypes.c_void_p(x.data_ptr()), (1 << 31) + 1,
                                                   None, None)
        assert mg.MagnusError(rc, "").name == "MAGNUS_ERR_WORKSPACE"
        # empty input: the total is 0
        tot = torch.full((1,), -7, dtype=torch.int64, device="cuda")
        rc = lib.magnus_exclusive_scan_i64_noalloc(ctx.handle, None, None, 0,
                                                   ctypes.c_void_p(tot.data_ptr()), None)
        assert rc == 0
        torch.cuda.synchronize()
        assert int(tot.item()) == 0
    finally:
        ctx.close()
