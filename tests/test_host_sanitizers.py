"""The repository's plain C++ under AddressSanitizer and
UndefinedBehaviorSanitizer (host only): the input generators and the oracle,
driven through their C entry points on small inputs of every index and value
width with several threads (tests/sanitize_main.cpp), and the admission
simulation of the serving loop (tests/admission_sim.cpp, which compiles the
server's admission rule).  Any memory error, leak or undefined behaviour
aborts the program."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1", "-std=c++17", "-pthread"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


def _build_and_run(tmp_path, name, srcs, extra=()):
    exe = str(tmp_path / name)
    r = subprocess.run(["g++", *SAN, *extra, *srcs, "-o", exe], capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower() and "cannot find" in r.stderr.lower():
        pytest.skip("the sanitizer runtimes are not installed")
    assert r.returncode == 0, r.stderr[-3000:]
    # the environment is passed on as it is; ASan is told not to insist on
    # being first among the preloaded libraries
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, (out.stdout[-2000:], out.stderr[-4000:])
    return out.stdout


def test_generators_and_oracle_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "sanitize_main",
                         [os.path.join(HERE, "sanitize_main.cpp"),
                          os.path.join(ROOT, "workloads", "gen.cpp"),
                          os.path.join(ROOT, "oracle", "oracle.cpp")],
                         extra=["-ffp-contract=off"])
    assert "total fails 0" in out


def test_admission_simulation_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "admission_sim", [os.path.join(HERE, "admission_sim.cpp")],
                         extra=["-I" + os.path.join(ROOT, "paper_2501_07056_amd", "csrc")])
    assert "mix " in out and "starvation " in out


def test_server_allocator_fuzz(tmp_path):
    """The serving loop's device-memory allocator (split best fit over slabs,
    merged on release): its source is taken from the serving code unchanged
    and exercised on the host with the HIP calls replaced."""
    src = open(os.path.join(ROOT, "paper_2501_07056_amd", "csrc", "server.hip")).read()
    i = src.index("struct DevCache {")
    j = src.index("void* srv_alloc(size_t n, void* stream, void* ctx) {")
    inc = tmp_path / "dev_cache.inc"
    inc.write_text(src[i:j])
    out = _build_and_run(tmp_path, "server_alloc_fuzz",
                         [os.path.join(HERE, "server_alloc_fuzz.cpp")],
                         extra=[f'-DDEVCACHE_SRC="{inc}"'])
    assert out.startswith("ok:"), out
