"""Python binding of the C ABI: torch tensors in and out, every step of the
product runs in the HIP library.  torch provides device memory (through the
library's allocator hook) and streams."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import (CsrDesc, CsrOutDesc, Options, PlanInfo, RequestInfo, ServerConfig, ServerStats,
                   check)

_ITYPE = {torch.int32: 0, torch.int64: 1}
_VTYPE = {torch.float32: 0, torch.float64: 1}
CATEGORY = {"auto": -1, "sort": 0, "dense": 1, "chunked": 2}


@dataclass
class DeviceCSR:
    """CSR matrix in device memory: rowptr (int32/int64), col (int32/int64),
    val (float32/float64)."""
    nrows: int
    ncols: int
    rowptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @classmethod
    def from_host(cls, M, device="cuda:0"):
        """From any object with nrows, ncols and numpy rowptr/col/val."""
        rp = torch.from_numpy(M.rowptr).to(device)
        col = torch.from_numpy(M.col).to(device)
        val = torch.from_numpy(M.val).to(device)
        return cls(int(M.nrows), int(M.ncols), rp, col, val)

    def desc(self) -> CsrDesc:
        d = CsrDesc()
        d.nrows, d.ncols, d.nnz = self.nrows, self.ncols, self.nnz
        d.rowptr_type = _ITYPE[self.rowptr.dtype]
        d.col_type = _ITYPE[self.col.dtype]
        d.val_type = _VTYPE[self.val.dtype]
        d.rowptr = self.rowptr.data_ptr()
        d.col = self.col.data_ptr() if self.col.numel() else None
        d.val = self.val.data_ptr() if self.val.numel() else None
        return d

    def to_host(self):
        return (self.rowptr.cpu().numpy(), self.col.cpu().numpy(), self.val.cpu().numpy())


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream), stream


class Context:
    """A library handle bound to one device, with torch's caching allocator
    behind the library's device allocations."""

    def __init__(self, device: int = 0, alloc_filter=None, **options):
        """alloc_filter: optional callable(nbytes) -> bool; an allocation it
        refuses is reported to the library as failed (the allocator returns
        NULL), so callers can exercise the library's out-of-memory paths.
        self.live_allocs counts allocations not yet freed."""
        self.lib = _lib.load()
        self.live_allocs = 0
        self.device = device
        self.handle = ctypes.c_void_p()
        self.opts = Options()
        self.lib.magnus_options_default(ctypes.byref(self.opts))
        self._apply(options)
        check(self.lib.magnus_create(ctypes.byref(self.handle), device, ctypes.byref(self.opts)),
              "magnus_create")
        dev = torch.device("cuda", device)

        def _alloc(n, stream, ctx):
            if alloc_filter is not None and not alloc_filter(int(n)):
                return None
            try:
                p = torch.cuda.caching_allocator_alloc(int(n), dev, int(stream or 0))
            except Exception:
                return None
            self.live_allocs += 1
            return p

        def _free(p, n, stream, ctx):
            self.live_allocs -= 1
            try:
                torch.cuda.caching_allocator_delete(int(p))
            except Exception:  # interpreter shutdown: torch already torn down
                pass

        self._alloc_cb = _lib.ALLOC_FN(_alloc)
        self._free_cb = _lib.FREE_FN(_free)
        check(self.lib.magnus_set_allocator(self.handle, self._alloc_cb, self._free_cb, None),
              "magnus_set_allocator")

    def _apply(self, options):
        for k, v in options.items():
            if k == "force_category" and isinstance(v, str):
                v = CATEGORY[v]
            if not hasattr(self.opts, k):
                raise TypeError(f"unknown option {k}")
            setattr(self.opts, k, int(v))

    def set_options(self, **options):
        self._apply(options)
        check(self.lib.magnus_set_options(self.handle, ctypes.byref(self.opts)),
              "magnus_set_options")

    def close(self):
        if self.handle:
            self.lib.magnus_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- calls
    def plan(self, A: DeviceCSR, B: DeviceCSR, stream=None) -> "Plan":
        s, keep = _stream_ptr(stream)
        da, db = A.desc(), B.desc()
        p = ctypes.c_void_p()
        info = PlanInfo()
        check(self.lib.magnus_plan(self.handle, ctypes.byref(da), ctypes.byref(db), s,
                                   ctypes.byref(p), ctypes.byref(info)), "magnus_plan",
              self.handle)
        return Plan(self, p, info, A, B)

    def row_ip(self, A: DeviceCSR, B: DeviceCSR, stream=None):
        s, keep = _stream_ptr(stream)
        out = torch.empty(max(A.nrows, 1), dtype=torch.int64, device=A.rowptr.device)
        tot = ctypes.c_int64()
        da, db = A.desc(), B.desc()
        check(self.lib.magnus_row_ip(self.handle, ctypes.byref(da), ctypes.byref(db),
                                     ctypes.c_void_p(out.data_ptr()), ctypes.byref(tot), s),
              "magnus_row_ip", self.handle)
        return out[:A.nrows], tot.value

    def exclusive_scan(self, x: torch.Tensor, stream=None):
        s, keep = _stream_ptr(stream)
        assert x.dtype == torch.int64 and x.is_contiguous()
        out = torch.empty_like(x)
        tot = ctypes.c_int64()
        check(self.lib.magnus_exclusive_scan_i64(
            self.handle, ctypes.c_void_p(x.data_ptr()) if x.numel() else None,
            ctypes.c_void_p(out.data_ptr()) if x.numel() else None, x.numel(), ctypes.byref(tot),
            s), "magnus_exclusive_scan_i64", self.handle)
        return out, tot.value

    def profile(self, on: bool = True):
        check(self.lib.magnus_profile_enable(self.handle, 1 if on else 0), "magnus_profile_enable")

    def profile_read(self):
        """Per-kernel launches, event milliseconds and algorithmic bytes since
        the last read (waits for the recorded events)."""
        arr = (_lib.KernelStat * 64)()
        n = ctypes.c_int32()
        check(self.lib.magnus_profile_read(self.handle, arr, 64, ctypes.byref(n)),
              "magnus_profile_read", self.handle)
        return [{"name": arr[i].name.decode(), "launches": int(arr[i].launches),
                 "ms": float(arr[i].ms), "bytes": float(arr[i].bytes)} for i in range(n.value)]

    def stream_copy(self, dst: torch.Tensor, src: torch.Tensor, stream=None):
        s, keep = _stream_ptr(stream)
        nbytes = src.numel() * src.element_size()
        assert dst.numel() * dst.element_size() >= nbytes
        check(self.lib.magnus_stream_copy(self.handle, ctypes.c_void_p(dst.data_ptr()),
                                          ctypes.c_void_p(src.data_ptr()), nbytes, s),
              "magnus_stream_copy", self.handle)

    def stream_copy_raw(self, dst: int, src: int, nbytes: int, stream=None):
        s, keep = _stream_ptr(stream)
        check(self.lib.magnus_stream_copy(self.handle, ctypes.c_void_p(dst), ctypes.c_void_p(src),
                                          nbytes, s), "magnus_stream_copy", self.handle)

    def stream_chunks(self, cols: torch.Tensor, vals: torch.Tensor, m: int, chunk_shift: int,
                      dense_min: int = 0, stream=None):
        """The chunk building blocks on one stream of products (Section 4.1):
        cols (device int32, each in [0, m)) and vals (device f32/f64).
        Returns the distinct columns (ascending), their sums and the per-stage
        event times."""
        s, keep = _stream_ptr(stream)
        assert cols.dtype == torch.int32 and cols.is_contiguous() and vals.is_contiguous()
        assert vals.dtype in (torch.float32, torch.float64) and vals.numel() == cols.numel()
        n = cols.numel()
        out_c = torch.empty(max(n, 1), dtype=torch.int32, device=cols.device)
        out_v = torch.empty(max(n, 1), dtype=vals.dtype, device=cols.device)
        nnz = ctypes.c_int64()
        t = _lib.StreamTimes()
        vt = 1 if vals.dtype == torch.float64 else 0
        check(self.lib.magnus_stream_chunks(
            self.handle, ctypes.c_void_p(cols.data_ptr()) if n else None,
            ctypes.c_void_p(vals.data_ptr()) if n else None, vt, n, int(m), int(chunk_shift),
            int(dense_min), ctypes.c_void_p(out_c.data_ptr()), ctypes.c_void_p(out_v.data_ptr()),
            ctypes.byref(nnz), s, ctypes.byref(t)), "magnus_stream_chunks", self.handle)
        return out_c[:nnz.value], out_v[:nnz.value], t.as_dict()

    def batch_plan(self, pairs, sort_max=None, stream=None) -> "BatchPlan":
        """Plan C_b = A_b * B_b for every (A_b, B_b) in pairs as one batch.
        sort_max: optional per-product SORT thresholds."""
        s, keep = _stream_ptr(stream)
        n = len(pairs)
        da = (CsrDesc * n)(*[a.desc() for a, _ in pairs])
        db = (CsrDesc * n)(*[b.desc() for _, b in pairs])
        sm = None
        if sort_max is not None:
            assert len(sort_max) == n
            sm = (ctypes.c_int32 * n)(*[int(x) for x in sort_max])
        nnz = (ctypes.c_int64 * n)()
        p = ctypes.c_void_p()
        info = PlanInfo()
        check(self.lib.magnus_batch_plan(self.handle, n, da, db, sm, s, ctypes.byref(p), nnz,
                                         ctypes.byref(info)), "magnus_batch_plan", self.handle)
        return BatchPlan(self, p, info, list(pairs), [int(x) for x in nnz])

    def batch_bound(self, pairs, stream=None):
        """(ip, nnz upper bound) of every product of the batch (host lists)."""
        s, keep = _stream_ptr(stream)
        n = len(pairs)
        da = (CsrDesc * n)(*[a.desc() for a, _ in pairs])
        db = (CsrDesc * n)(*[b.desc() for _, b in pairs])
        ip, nb = (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)()
        check(self.lib.magnus_batch_bound(self.handle, n, da, db, s, ip, nb), "magnus_batch_bound",
              self.handle)
        return list(ip), list(nb)

    def spgemm(self, A: DeviceCSR, B: DeviceCSR, rowptr_dtype=torch.int64, stream=None):
        """C = A*B into torch-owned tensors (plan, execute, destroy)."""
        p = self.plan(A, B, stream)
        try:
            return p.execute(rowptr_dtype=rowptr_dtype, stream=stream)
        finally:
            p.destroy()

    def spgemm_lib(self, A: DeviceCSR, B: DeviceCSR, rowptr_dtype=torch.int64, stream=None):
        """C = A*B by the C ABI's one-call product (magnus_spgemm): C comes
        from the library's allocator, i.e. torch's caching allocator here.
        Returns a LibCSR that owns that memory until free() (or collection)."""
        s, keep = _stream_ptr(stream)
        da, db = A.desc(), B.desc()
        d = CsrOutDesc()
        check(self.lib.magnus_spgemm(self.handle, ctypes.byref(da), ctypes.byref(db),
                                     _ITYPE[rowptr_dtype], ctypes.byref(d), s),
              "magnus_spgemm", self.handle)
        return LibCSR(self, d)


class LibCSR:
    """A C whose arrays the library allocated (magnus_spgemm); free() hands
    them back through magnus_csr_free."""

    def __init__(self, ctx: Context, d: CsrOutDesc):
        self.ctx, self.d = ctx, d

    @property
    def nnz(self) -> int:
        return int(self.d.capacity)

    def to_device_csr(self) -> DeviceCSR:
        """A copy into torch-owned tensors (by the library's copy kernel)."""
        d = self.d
        dev = torch.device("cuda", self.ctx.device)
        rt = torch.int64 if d.rowptr_type == 1 else torch.int32
        ct = torch.int64 if d.col_type == 1 else torch.int32
        vt = torch.float64 if d.val_type == 1 else torch.float32
        out = DeviceCSR(int(d.nrows), int(d.ncols),
                        torch.empty(int(d.nrows) + 1, dtype=rt, device=dev),
                        torch.empty(self.nnz, dtype=ct, device=dev),
                        torch.empty(self.nnz, dtype=vt, device=dev))
        for t, src in ((out.rowptr, d.rowptr), (out.col, d.col), (out.val, d.val)):
            if t.numel():
                self.ctx.stream_copy_raw(t.data_ptr(), src, t.numel() * t.element_size())
        return out

    def free(self, stream=None):
        if self.d is not None and self.ctx.handle:
            s, keep = _stream_ptr(stream)
            check(self.ctx.lib.magnus_csr_free(self.ctx.handle, ctypes.byref(self.d), s),
                  "magnus_csr_free")
        self.d = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Plan:
    def __init__(self, ctx: Context, ptr, info: PlanInfo, A, B):
        self.ctx, self.ptr, self.info, self.A, self.B = ctx, ptr, info, A, B

    @property
    def nnz(self) -> int:
        return int(self.info.nnz_c)

    def alloc_output(self, rowptr_dtype=torch.int64, capacity=None) -> DeviceCSR:
        dev = self.A.rowptr.device
        cap = self.nnz if capacity is None else capacity
        return DeviceCSR(self.A.nrows, self.B.ncols,
                         torch.empty(self.A.nrows + 1, dtype=rowptr_dtype, device=dev),
                         torch.empty(max(cap, 0), dtype=self.B.col.dtype, device=dev),
                         torch.empty(max(cap, 0), dtype=self.A.val.dtype, device=dev))

    def execute(self, C: DeviceCSR | None = None, rowptr_dtype=torch.int64, stream=None):
        s, keep = _stream_ptr(stream)
        if C is None:
            C = self.alloc_output(rowptr_dtype)
        d = _out_desc(C)
        nnz = ctypes.c_int64()
        da, db = self.A.desc(), self.B.desc()
        check(self.ctx.lib.magnus_execute(self.ctx.handle, self.ptr, ctypes.byref(da),
                                          ctypes.byref(db), ctypes.byref(d), ctypes.byref(nnz), s),
              "magnus_execute", self.ctx.handle)
        return C

    def destroy(self):
        if self.ptr:
            self.ctx.lib.magnus_plan_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _out_desc(C: DeviceCSR) -> CsrOutDesc:
    d = CsrOutDesc()
    d.nrows, d.ncols, d.capacity = C.nrows, C.ncols, C.col.numel()
    d.rowptr_type = _ITYPE[C.rowptr.dtype]
    d.col_type = _ITYPE[C.col.dtype]
    d.val_type = _VTYPE[C.val.dtype]
    d.rowptr = C.rowptr.data_ptr()
    d.col = C.col.data_ptr() if C.col.numel() else None
    d.val = C.val.data_ptr() if C.val.numel() else None
    return d


class BatchPlan:
    """A planned batch: nnz[b] is nnz(C_b); execute() runs the numeric phase
    of every product (captured into a HIP graph on the first call, replayed
    afterwards, unless graph=False)."""

    def __init__(self, ctx: Context, ptr, info: PlanInfo, pairs, nnz):
        self.ctx, self.ptr, self.info, self.pairs, self.nnz = ctx, ptr, info, pairs, nnz

    def alloc_outputs(self, rowptr_dtype=torch.int64):
        outs = []
        for (A, B), nz in zip(self.pairs, self.nnz):
            dev = A.rowptr.device
            outs.append(DeviceCSR(A.nrows, B.ncols,
                                  torch.empty(A.nrows + 1, dtype=rowptr_dtype, device=dev),
                                  torch.empty(nz, dtype=B.col.dtype, device=dev),
                                  torch.empty(nz, dtype=A.val.dtype, device=dev)))
        return outs

    def execute(self, outs=None, rowptr_dtype=torch.int64, graph: bool = True, stream=None,
                pairs=None, persistent: bool = False):
        s, keep = _stream_ptr(stream)
        pairs = self.pairs if pairs is None else pairs
        if outs is None:
            outs = self.alloc_outputs(rowptr_dtype)
        n = len(pairs)
        da = (CsrDesc * n)(*[a.desc() for a, _ in pairs])
        db = (CsrDesc * n)(*[b.desc() for _, b in pairs])
        dc = (CsrOutDesc * n)(*[_out_desc(C) for C in outs])
        mode = _lib.BATCH_GRAPH if graph else _lib.BATCH_EAGER
        if persistent:
            mode |= _lib.BATCH_PERSISTENT
        check(self.ctx.lib.magnus_batch_execute(self.ctx.handle, self.ptr, n, da, db, dc, mode, s),
              "magnus_batch_execute", self.ctx.handle)
        return outs

    def destroy(self):
        if self.ptr:
            self.ctx.lib.magnus_batch_plan_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


REQ_STATE = {0: "queued", 1: "running", 2: "done", 3: "rejected", 4: "failed"}


class Server:
    """Request loop over device-resident operands (see magnus_server_* in
    include/magnus.h).  register() keeps a reference to each operand so its
    device memory outlives the server."""

    def __init__(self, device: int = 0, options=None, **config):
        self.lib = _lib.load()
        self.device = device
        opts = Options()
        self.lib.magnus_options_default(ctypes.byref(opts))
        for k, v in (options or {}).items():
            if k == "force_category" and isinstance(v, str):
                v = CATEGORY[v]
            setattr(opts, k, int(v))
        cfg = ServerConfig()
        self.lib.magnus_server_config_default(ctypes.byref(cfg))
        for k, v in config.items():
            if not hasattr(cfg, k):
                raise TypeError(f"unknown server setting {k}")
            setattr(cfg, k, int(v))
        self.ptr = ctypes.c_void_p()
        check(self.lib.magnus_server_create(device, ctypes.byref(opts), ctypes.byref(cfg),
                                            ctypes.byref(self.ptr)), "magnus_server_create")
        self.ops = []
        self._copier = None

    def register(self, X: DeviceCSR) -> int:
        i = ctypes.c_int32()
        d = X.desc()
        check(self.lib.magnus_server_register(self.ptr, ctypes.byref(d), ctypes.byref(i)),
              "magnus_server_register")
        self.ops.append(X)
        return i.value

    def submit(self, a_id: int, b_id: int) -> int:
        r = ctypes.c_int64()
        check(self.lib.magnus_server_submit(self.ptr, a_id, b_id, ctypes.byref(r)),
              "magnus_server_submit")
        return r.value

    def query(self, rid: int) -> dict:
        info = RequestInfo()
        check(self.lib.magnus_server_query(self.ptr, rid, ctypes.byref(info)), "magnus_server_query")
        d = {n: getattr(info, n) for n, _ in info._fields_ if n != "_pad"}
        d["state"] = REQ_STATE[d["state"]]
        return d

    def ready(self, rid: int) -> bool:
        return self.query(rid)["state"] in ("done", "rejected", "failed")

    def result(self, rid: int) -> DeviceCSR:
        """C of a finished request, copied by the library's copy kernel into
        tensors that torch owns (the server's memory is freed by release)."""
        d = CsrOutDesc()
        check(self.lib.magnus_server_result(self.ptr, rid, ctypes.byref(d)), "magnus_server_result")
        if self._copier is None:
            self._copier = Context(self.device)
        dev = self.ops[0].rowptr.device
        nnz = int(d.capacity)
        ct = torch.int64 if d.col_type == 1 else torch.int32
        vt = torch.float64 if d.val_type == 1 else torch.float32
        out = DeviceCSR(int(d.nrows), int(d.ncols),
                        torch.empty(int(d.nrows) + 1, dtype=torch.int64, device=dev),
                        torch.empty(nnz, dtype=ct, device=dev), torch.empty(nnz, dtype=vt, device=dev))
        lib, h = self._copier.lib, self._copier.handle
        s = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
        for t, src in ((out.rowptr, d.rowptr), (out.col, d.col), (out.val, d.val)):
            if t.numel():
                check(lib.magnus_stream_copy(h, ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(src),
                                             t.numel() * t.element_size(), s), "magnus_stream_copy")
        # the copies read the server's memory: finish them before a release
        # can hand that memory to another request
        torch.cuda.current_stream(dev).synchronize()
        return out

    def result_rows(self, rid: int, rows):
        """Row pointers of a finished request's C and the columns and values
        of the given rows only, as host arrays (rowptr, col, val; col and val
        concatenated in the order of rows), read from the server's memory
        without copying C whole."""
        import numpy as np
        d = CsrOutDesc()
        check(self.lib.magnus_server_result(self.ptr, rid, ctypes.byref(d)), "magnus_server_result")
        if self._copier is None:
            self._copier = Context(self.device)
        dev = self.ops[0].rowptr.device
        cb = 8 if d.col_type == 1 else 4
        vb = 8 if d.val_type == 1 else 4
        ct = torch.int64 if cb == 8 else torch.int32
        vt = torch.float64 if vb == 8 else torch.float32
        lib, h = self._copier.lib, self._copier.handle
        s = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)

        def copy(dst: torch.Tensor, src: int, nbytes: int):
            if nbytes:
                check(lib.magnus_stream_copy(h, ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src),
                                             nbytes, s), "magnus_stream_copy")
        rp_d = torch.empty(int(d.nrows) + 1, dtype=torch.int64, device=dev)
        copy(rp_d, d.rowptr, rp_d.numel() * 8)
        rp = rp_d.cpu().numpy()
        rows = np.asarray(rows, dtype=np.int64)
        lens = rp[rows + 1] - rp[rows]
        tot = int(lens.sum())
        col = torch.empty(tot, dtype=ct, device=dev)
        val = torch.empty(tot, dtype=vt, device=dev)
        o = 0
        for r, ln in zip(rows.tolist(), lens.tolist()):
            if ln:
                copy(col[o:], d.col + int(rp[r]) * cb, ln * cb)
                copy(val[o:], d.val + int(rp[r]) * vb, ln * vb)
            o += ln
        torch.cuda.current_stream(dev).synchronize()
        return rp, col.cpu().numpy(), val.cpu().numpy()

    def poll(self, max_n: int = 64):
        """Final states reported since the last poll: a list of dicts
        (request_id, state, status, nnz, latency_ms)."""
        arr = (_lib.Completion * max_n)()
        n = ctypes.c_int32()
        check(self.lib.magnus_server_poll(self.ptr, arr, max_n, ctypes.byref(n)),
              "magnus_server_poll")
        return [{"request_id": arr[i].request_id, "state": REQ_STATE[arr[i].state],
                 "status": arr[i].status, "nnz": arr[i].nnz, "latency_ms": arr[i].latency_ms}
                for i in range(n.value)]

    def release(self, rid: int):
        check(self.lib.magnus_server_release(self.ptr, rid), "magnus_server_release")

    def stats(self) -> dict:
        st = ServerStats()
        check(self.lib.magnus_server_get_stats(self.ptr, ctypes.byref(st)), "magnus_server_get_stats")
        return {n: getattr(st, n) for n, _ in st._fields_}

    def close(self):
        if self.ptr:
            self.lib.magnus_server_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()
        if self._copier is not None:
            self._copier.close()
            self._copier = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def paper_chunk_model(m_c: int, s_cache: int, s_line: int, s_dense_accum: float):
    """Eqs. 2-7 (host only): (n_chunks_fine, n_chunks_coarse, m_CmaxL2)."""
    lib = _lib.load()
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    check(lib.magnus_paper_chunk_model(m_c, s_cache, s_line, float(s_dense_accum),
                                       ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
          "magnus_paper_chunk_model")
    return a.value, b.value, c.value


def gpu_chunk_shift(f64: bool, lds_bytes: int) -> int:
    lib = _lib.load()
    s = ctypes.c_int32()
    check(lib.magnus_gpu_chunk_shift(1 if f64 else 0, lds_bytes, ctypes.byref(s)),
          "magnus_gpu_chunk_shift")
    return s.value
