"""Host-side checks of the HIP library (no GPU needed): it loads, exports
every call include/magnus.h declares, validates arguments before touching a
device, and its host-only model functions agree with the oracle's."""
import ctypes
import os

import pytest

import paper_2501_07056_amd as mg
from paper_2501_07056_amd import _lib
from oracle import chunk_model as cm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    lib = mg.load()
    names = mg.declared_symbols()
    for must in ("magnus_plan", "magnus_execute", "magnus_batch_plan", "magnus_batch_execute",
                 "magnus_batch_bound", "magnus_server_create", "magnus_server_submit",
                 "magnus_server_result", "magnus_server_release", "magnus_row_ip"):
        assert must in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_cover_the_enum():
    lib = mg.load()
    for code, name in _lib.STATUS.items():
        assert lib.magnus_status_string(code).decode() == name
    assert lib.magnus_status_string(999).decode() == "MAGNUS_ERR_UNKNOWN"


def test_defaults_are_model_choices():
    o = _lib.Options()
    mg.load().magnus_options_default(ctypes.byref(o))
    assert o.force_category == -1
    for f in ("sort_max", "chunk_shift", "bin_dense_min", "tile_products", "dense_block",
              "batch_products", "max_workspace_bytes", "validate", "lds_bytes", "deterministic"):
        assert getattr(o, f) == 0, f


def test_options_layout_matches_the_header():
    """The deterministic and chunk_runs fields took reserved words: the
    struct keeps its size, and the fields sit where the header puts them."""
    hdr = open(os.path.join(ROOT, "include", "magnus.h")).read()
    body = hdr[hdr.index("typedef struct {\n  int32_t force_category;"):]
    body = body[:body.index("} magnus_options_t;")]
    assert "int32_t deterministic;" in body and "int32_t chunk_runs;" in body
    assert "int32_t _reserved;" in body
    assert ctypes.sizeof(_lib.Options) == 72
    assert _lib.Options.deterministic.offset == _lib.Options.coarse_chunks.offset + 4
    assert _lib.Options.chunk_runs.offset == _lib.Options.deterministic.offset + 4


def test_deterministic_server_rejected_before_any_device_call():
    o = _lib.Options()
    lib = mg.load()
    lib.magnus_options_default(ctypes.byref(o))
    o.deterministic = 1
    out = ctypes.c_void_p()
    assert lib.magnus_server_create(0, ctypes.byref(o), None, ctypes.byref(out)) == 1


def test_null_arguments_rejected_before_any_device_call():
    lib = mg.load()
    INVALID = 1
    assert lib.magnus_plan(None, None, None, None, None, None) == INVALID
    assert lib.magnus_execute(None, None, None, None, None, None, None) == INVALID
    assert lib.magnus_batch_plan(None, 0, None, None, None, None, None, None, None) == INVALID
    assert lib.magnus_batch_execute(None, None, 0, None, None, None, 0, None) == INVALID
    assert lib.magnus_batch_bound(None, 0, None, None, None, None, None) == INVALID
    assert lib.magnus_server_create(0, None, None, None) == INVALID
    assert lib.magnus_server_submit(None, 0, 0, None) == INVALID
    assert lib.magnus_server_release(None, 1) == INVALID
    assert lib.magnus_stream_chunks(None, None, None, 0, 0, 1, 4, 0, None, None, None, None,
                                    None) == INVALID
    assert lib.magnus_plan_destroy(None) == 0
    assert lib.magnus_batch_plan_destroy(None) == 0
    assert lib.magnus_server_destroy(None) == 0
    cfg = _lib.ServerConfig()
    cfg.max_batch = -1
    out = ctypes.c_void_p()
    assert lib.magnus_server_create(0, None, ctypes.byref(cfg), ctypes.byref(out)) == INVALID


@pytest.mark.parametrize("s_val", [4, 8])
@pytest.mark.parametrize("phase", ["numeric", "symbolic"])
def test_library_chunk_model_matches_oracle(s_val, phase):
    """magnus_paper_chunk_model evaluates Eqs. 2-7 like the oracle over a
    sweep of matrix widths, cache sizes and line sizes."""
    sd = (s_val + 1) if phase == "numeric" else 1
    for s_l2 in (32 << 10, 160 << 10, 1 << 20, 4 << 20):
        for line in (64, 128):
            for lg in range(0, 31, 3):
                m = (1 << lg) + (lg % 2)
                ref = cm.paper_model(m, s_l2, line, s_val, phase)
                got = mg.paper_chunk_model(m, s_l2, line, sd)
                assert got == (ref["n_chunks_fine"], ref["n_chunks_coarse"], ref["m_cmax"]), \
                    (m, s_l2, line, got, ref)


def test_gpu_chunk_shift_fits_lds():
    """The chunk length's dense accumulator (value plus one bitmap bit per
    column) takes at most half of the LDS budget, and the next power of two
    would not fit; 16 is the cap (16-bit chunk-local columns)."""
    for f64, sv in ((True, 8.0), (False, 4.0)):
        prev = 0
        for lds in (16 << 10, 32 << 10, 64 << 10, 160 << 10, 1 << 20):
            s = mg.gpu_chunk_shift(f64, lds)
            per = sv + 0.125
            assert per * (1 << s) + 1024 <= lds / 2 or s == 8
            assert s == 16 or per * (1 << (s + 1)) + 1024 > lds / 2
            assert s >= prev
            prev = s
    assert mg.gpu_chunk_shift(True, 160 << 10) == 13
    assert mg.gpu_chunk_shift(False, 160 << 10) == 14
    with pytest.raises(mg.MagnusError):
        mg.gpu_chunk_shift(True, 0)
