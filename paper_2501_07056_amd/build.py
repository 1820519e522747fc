"""Build the gfx950 HIP library in-tree: every csrc/*.hip is compiled by hipcc
in parallel and linked into paper_2501_07056_amd/libmagnus.so.  The checked
build (checked=True) compiles the same sources with MG_CHECKED into
libmagnus_checked.so: guard bytes around every plan allocation, verified
after each plan and each numeric phase."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmagnus.so")
OUT_CHECKED = os.path.join(HERE, "libmagnus_checked.so")
OBJ = os.path.join(ROOT, "_build")
# extra compiler flags and an alternative output, for experiment builds
EXTRA = os.environ.get("MAGNUS_EXTRA_FLAGS", "").split()
if os.environ.get("MAGNUS_LIB_OUT"):
    OUT = os.path.abspath(os.environ["MAGNUS_LIB_OUT"])
    OBJ = OUT + ".objs"
ARCH = os.environ.get("MAGNUS_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
         # packed fp32 instructions are left to nobody: keep them out of codegen
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"] + EXTRA


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    return "hipcc"


def _compile(src: str, force: bool, objdir: str, flags: list) -> str:
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    deps = [src] + glob.glob(os.path.join(CSRC, "*.h")) + [os.path.join(ROOT, "include", "magnus.h")]
    if not force and os.path.exists(obj) and os.path.getmtime(obj) >= max(os.path.getmtime(d) for d in deps):
        return obj
    cmd = [_hipcc()] + flags + ["-c", src, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    os.replace(obj + ".tmp", obj)
    return obj


def build(force: bool = True, jobs: int | None = None, verbose: bool = False,
          checked: bool = False) -> str:
    out = OUT_CHECKED if checked else OUT
    objdir = os.path.join(OBJ, "checked") if checked else OBJ
    flags = FLAGS + (["-DMG_CHECKED"] if checked else [])
    os.makedirs(objdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force, objdir, flags), srcs))
    tmp = out + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(force="--force" in sys.argv, verbose=True, checked="--checked" in sys.argv)
