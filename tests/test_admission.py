"""The serving loop's admission rule (the header the server compiles),
driven by a host simulation with a fake executor: no deadlock, C memory
within the budget, rejection only of requests that cannot fit even when
sized exactly, and a large request is not passed by small ones forever."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2501_07056_amd", "csrc")


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sim") / "admission_sim")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror", "-I" + CSRC,
                    os.path.join(HERE, "admission_sim.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in out.splitlines():
        name, comp, rej, dead, over, waits = line.split()
        res[name] = dict(completed=int(comp), rejected=int(rej), deadlock=int(dead),
                         c_over_budget=int(over), max_wait=int(waits))
    return res


def test_mix_completes_within_budget(sim):
    r = sim["mix"]
    assert r["deadlock"] == 0 and r["rejected"] == 0 and r["completed"] == 400
    assert r["c_over_budget"] <= 0


def test_exact_sizing_above_a_quarter_of_the_budget(sim):
    """Requests whose bounds exceed a quarter of the budget are sized exactly
    before admission (their bounds alone would fit): the mix still completes
    within the budget, without rejections."""
    r = sim["mix_quarter"]
    assert r["deadlock"] == 0 and r["rejected"] == 0 and r["completed"] == 400
    assert r["c_over_budget"] <= 0


def test_oversized_requests_each_fitting_alone(sim):
    """Several requests whose bounds exceed the budget and whose exact sizes
    fit only one at a time: all are served, one after another."""
    r = sim["oversized_pair"]
    assert r["deadlock"] == 0 and r["completed"] == 6 and r["c_over_budget"] <= 0


def test_reject_only_what_never_fits(sim):
    r = sim["reject_one"]
    assert r["rejected"] == 1 and r["completed"] == 29 and r["deadlock"] == 0


def test_large_request_not_starved(sim):
    r = sim["starvation"]
    assert r["completed"] == 2000 and r["deadlock"] == 0 and r["c_over_budget"] <= 0
