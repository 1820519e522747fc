"""The checked build of the library (MG_CHECKED: guard bytes around every
plan allocation, verified after each plan, numeric phase and batch execute;
an overwrite returns MAGNUS_ERR_INTERNAL) runs the single-product paths
(runs and product binning, the coarse level, SORT and DENSE rows) and a
batch with a CHUNKED product, eager and through the graph, against the
oracle, in a process of its own (tests/checked_cases.py)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(os.path.dirname(HERE), "paper_2501_07056_amd", "libmagnus_checked.so")


def test_checked_build_guards_hold():
    if not os.path.exists(LIB):
        pytest.skip("libmagnus_checked.so not built")
    env = dict(os.environ, MAGNUS_LIB=LIB)
    out = subprocess.run([sys.executable, "-u", os.path.join(HERE, "checked_cases.py")],
                         capture_output=True, text=True, env=env, timeout=240)
    print(out.stdout[-3000:])
    assert out.returncode == 0, (out.stdout[-2000:], out.stderr[-4000:])
    assert "checked cases ok" in out.stdout
