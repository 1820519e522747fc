"""ctypes declarations of the C ABI in include/magnus.h (marshalling only)."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmagnus.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "magnus.h")

c_i64 = ctypes.c_int64
c_i32 = ctypes.c_int32
c_vp = ctypes.c_void_p


class CsrDesc(ctypes.Structure):
    _fields_ = [("nrows", c_i64), ("ncols", c_i64), ("nnz", c_i64),
                ("rowptr_type", c_i32), ("col_type", c_i32), ("val_type", c_i32), ("_pad", c_i32),
                ("rowptr", c_vp), ("col", c_vp), ("val", c_vp)]


class CsrOutDesc(ctypes.Structure):
    _fields_ = [("nrows", c_i64), ("ncols", c_i64), ("capacity", c_i64),
                ("rowptr_type", c_i32), ("col_type", c_i32), ("val_type", c_i32), ("_pad", c_i32),
                ("rowptr", c_vp), ("col", c_vp), ("val", c_vp)]


class Options(ctypes.Structure):
    _fields_ = [("force_category", c_i32), ("sort_max", c_i32), ("chunk_shift", c_i32),
                ("bin_dense_min", c_i32), ("tile_products", c_i32), ("dense_block", c_i32),
                ("batch_products", c_i64), ("max_workspace_bytes", c_i64), ("validate", c_i32),
                ("lds_bytes", c_i32), ("sort_group_max", c_i32), ("stream_hints", c_i32),
                ("coarse_chunks", c_i32), ("deterministic", c_i32), ("chunk_runs", c_i32),
                ("_reserved", c_i32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("ip_total", c_i64), ("flops", c_i64), ("nnz_c", c_i64), ("max_row_ip", c_i64),
                ("rows_by_category", c_i64 * 4), ("ip_by_category", c_i64 * 4),
                ("nnz_by_category", c_i64 * 4),
                ("n_batches", c_i64), ("n_bins", c_i64), ("n_dense_chunks", c_i64),
                ("n_sort_groups", c_i64), ("plan_bytes", c_i64),
                ("chunk_shift", c_i32), ("sort_max", c_i32), ("bin_dense_min", c_i32),
                ("tile_products", c_i32), ("symbolic_ms", ctypes.c_double),
                ("coarse_rows", c_i64), ("coarse_chunks", c_i64), ("coarse_fine_chunks", c_i64),
                ("coarse_shift", c_i32), ("run_binned", c_i32), ("n_runs", c_i64)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if isinstance(v, ctypes.Array) else v
        return d


class ServerConfig(ctypes.Structure):
    _fields_ = [("memory_budget_bytes", c_i64), ("workspace_cap_bytes", c_i64),
                ("max_inflight", c_i32), ("max_batch", c_i32), ("streams", c_i32),
                ("max_bypass", c_i32), ("plan_estimate_pct", c_i32), ("exact_above_pct", c_i32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("state", c_i32), ("batch_size", c_i32), ("nnz", c_i64), ("bound_bytes", c_i64),
                ("exact_bytes", c_i64), ("queue_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double), ("status", c_i32), ("_pad", c_i32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, c_i64) for n in ("submitted", "completed", "rejected", "failed", "batches",
                                     "batched_requests", "exact_probes", "reserved_bytes",
                                     "budget_bytes", "queued", "running",
                                     "peak_reserved_bytes", "deferred")]


class Completion(ctypes.Structure):
    _fields_ = [("request_id", c_i64), ("state", c_i32), ("status", c_i32), ("nnz", c_i64),
                ("latency_ms", ctypes.c_double)]


class StreamTimes(ctypes.Structure):
    _fields_ = [("histogram_ms", ctypes.c_double), ("scan_ms", ctypes.c_double),
                ("reorder_ms", ctypes.c_double), ("group_ms", ctypes.c_double),
                ("count_ms", ctypes.c_double), ("accumulate_ms", ctypes.c_double),
                ("chunks", c_i64), ("dense_chunks", c_i64), ("sort_groups", c_i64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", c_i64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(c_vp, ctypes.c_size_t, c_vp, c_vp)
FREE_FN = ctypes.CFUNCTYPE(None, c_vp, ctypes.c_size_t, c_vp, c_vp)

BATCH_GRAPH = 0
BATCH_EAGER = 1
BATCH_PERSISTENT = 2

STATUS = {}
_lib = None


def _parse_status():
    src = open(HEADER).read()
    for name, val in re.findall(r"(MAGNUS_(?:OK|ERR_[A-Z_]+))\s*=\s*(\d+)", src):
        STATUS[int(val)] = name


def declared_symbols():
    """Function names declared in include/magnus.h."""
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(magnus_[a-z0-9_]+)\s*\(", src)))


def load(path: str = LIB_PATH):
    """Load the built library; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    # an alternative build of the same sources (A/B timing of compile-time
    # variants) may be named by MAGNUS_LIB
    path = os.environ.get("MAGNUS_LIB", path)
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.magnus_status_string.argtypes = [c_i32]
    lib.magnus_status_string.restype = ctypes.c_char_p
    lib.magnus_last_error.argtypes = [c_vp]
    lib.magnus_last_error.restype = ctypes.c_char_p
    lib.magnus_options_default.argtypes = [P(Options)]
    lib.magnus_options_default.restype = None
    lib.magnus_create.argtypes = [P(c_vp), c_i32, P(Options)]
    lib.magnus_destroy.argtypes = [c_vp]
    lib.magnus_set_options.argtypes = [c_vp, P(Options)]
    lib.magnus_set_allocator.argtypes = [c_vp, ALLOC_FN, FREE_FN, c_vp]
    lib.magnus_plan.argtypes = [c_vp, P(CsrDesc), P(CsrDesc), c_vp, P(c_vp), P(PlanInfo)]
    lib.magnus_execute.argtypes = [c_vp, c_vp, P(CsrDesc), P(CsrDesc), P(CsrOutDesc), P(c_i64),
                                   c_vp]
    lib.magnus_plan_destroy.argtypes = [c_vp]
    lib.magnus_spgemm.argtypes = [c_vp, P(CsrDesc), P(CsrDesc), c_i32, P(CsrOutDesc), c_vp]
    lib.magnus_csr_free.argtypes = [c_vp, P(CsrOutDesc), c_vp]
    lib.magnus_plan_get_info.argtypes = [c_vp, P(PlanInfo)]
    lib.magnus_row_ip.argtypes = [c_vp, P(CsrDesc), P(CsrDesc), c_vp, P(c_i64), c_vp]
    lib.magnus_paper_chunk_model.argtypes = [c_i64, c_i64, c_i64, ctypes.c_double, P(c_i64),
                                             P(c_i64), P(c_i64)]
    lib.magnus_gpu_chunk_shift.argtypes = [c_i32, c_i64, P(c_i32)]
    lib.magnus_exclusive_scan_i64.argtypes = [c_vp, c_vp, c_vp, c_i64, P(c_i64), c_vp]
    lib.magnus_exclusive_scan_i64_noalloc.argtypes = [c_vp, c_vp, c_vp, c_i64, c_vp, c_vp]
    lib.magnus_profile_enable.argtypes = [c_vp, c_i32]
    lib.magnus_profile_read.argtypes = [c_vp, P(KernelStat), c_i32, P(c_i32)]
    lib.magnus_stream_copy.argtypes = [c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]
    lib.magnus_stream_chunks.argtypes = [c_vp, c_vp, c_vp, c_i32, c_i64, c_i64, c_i32, c_i32,
                                         c_vp, c_vp, P(c_i64), c_vp, P(StreamTimes)]
    lib.magnus_batch_plan.argtypes = [c_vp, c_i32, P(CsrDesc), P(CsrDesc), P(c_i32), c_vp,
                                      P(c_vp), P(c_i64), P(PlanInfo)]
    lib.magnus_batch_execute.argtypes = [c_vp, c_vp, c_i32, P(CsrDesc), P(CsrDesc),
                                         P(CsrOutDesc), c_i32, c_vp]
    lib.magnus_batch_plan_destroy.argtypes = [c_vp]
    lib.magnus_batch_bound.argtypes = [c_vp, c_i32, P(CsrDesc), P(CsrDesc), c_vp, P(c_i64),
                                       P(c_i64)]
    lib.magnus_server_config_default.argtypes = [P(ServerConfig)]
    lib.magnus_server_config_default.restype = None
    lib.magnus_server_create.argtypes = [c_i32, P(Options), P(ServerConfig), P(c_vp)]
    lib.magnus_server_destroy.argtypes = [c_vp]
    lib.magnus_server_register.argtypes = [c_vp, P(CsrDesc), P(c_i32)]
    lib.magnus_server_submit.argtypes = [c_vp, c_i32, c_i32, P(c_i64)]
    lib.magnus_server_query.argtypes = [c_vp, c_i64, P(RequestInfo)]
    lib.magnus_server_result.argtypes = [c_vp, c_i64, P(CsrOutDesc)]
    lib.magnus_server_release.argtypes = [c_vp, c_i64]
    lib.magnus_server_get_stats.argtypes = [c_vp, P(ServerStats)]
    lib.magnus_server_poll.argtypes = [c_vp, P(Completion), c_i32, P(c_i32)]
    for fn in declared_symbols():
        f = getattr(lib, fn)
        if fn not in ("magnus_status_string", "magnus_last_error", "magnus_options_default",
                      "magnus_server_config_default"):
            f.restype = c_i32
    _parse_status()
    _lib = lib
    return lib


class MagnusError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        self.name = STATUS.get(code, str(code))
        super().__init__(f"{where}: {self.name}" + (f" ({detail})" if detail else ""))


def check(code: int, where: str, handle=None):
    if code != 0:
        detail = ""
        if handle is not None and code == 10:
            detail = (load().magnus_last_error(handle) or b"").decode(errors="replace")
        raise MagnusError(code, where, detail)
