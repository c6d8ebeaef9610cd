"""CPU tests of the decode server's admission policy against a fake backend.

The policy (csrc/admit.h, the code the server runs) is compiled into a small simulator
(tests/admission_sim.cpp) whose launches complete after their estimated device time.
The simulator checks every invariant as it runs: chunks are taken from the front of the
queue in arrival order, each starts where its request's admission stopped, nothing
passes a partly admitted request, the budget in flight never exceeds the configured
bytes, own-launch chunks are alone and cut to their time target, ragged launches stop
at theirs, launches respect the codeword cap, per-request mode puts one chunk in each
launch, a failed launch drops only its requests, and every other request completes
whole.  Each scenario below also checks that its pressure really happened (requests
were split, slots overlapped, a request failed or was rejected).
"""
import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "admission_sim.cpp")
INC = os.path.join(ROOT, "paper_2508_03567_amd", "csrc")


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if not cxx:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("admission") / "admission_sim")
    subprocess.run([cxx, "-std=c++17", "-O2", "-Wall", "-Wextra", "-Werror", "-I", INC, SRC, "-o", exe], check=True)
    return exe


def _run(exe, seed, continuous, budget, slots, cap, nreq, spread, fail_at, target_us=None):
    args = [exe, str(seed), str(int(continuous)), str(budget), str(slots), str(cap), str(nreq), str(int(spread)),
            str(fail_at)]
    if target_us is not None:
        args.append(str(target_us))
    p = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, p.stderr
    return json.loads(p.stdout)


MiB = 1 << 20


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_continuous_large_budget(sim, seed):
    r = _run(sim, seed, True, 256 * MiB, 4, 0, 200, True, 0)
    assert r["failed"] == 0 and r["rejected"] == 0
    assert r["peak"] <= r["budget"]
    assert r["max_busy"] > 1  # launches overlapped
    assert r["chunks"] >= r["launches"]


@pytest.mark.parametrize("seed", [4, 5])
def test_small_budget_splits_requests(sim, seed):
    r = _run(sim, seed, True, 16 * MiB, 3, 96, 200, False, 0)
    assert r["split"] > 0 and r["peak"] <= r["budget"]
    assert r["launches"] > r["requests"]


def test_per_request_mode(sim):
    r = _run(sim, 6, False, 256 * MiB, 4, 0, 100, True, 0)
    assert r["launches"] == r["chunks"] and r["max_busy"] == 1


@pytest.mark.parametrize("target_us", [20, 40])
def test_ragged_launch_time_target(sim, target_us):
    r = _run(sim, 7, True, 256 * MiB, 4, 0, 300, False, 0, target_us)
    assert r["launches"] > 1 and r["chunks"] > r["launches"]


@pytest.mark.parametrize("fail_at", [3, 5])
def test_failed_launch_drops_only_its_requests(sim, fail_at):
    r = _run(sim, 8 + fail_at, True, 30 * MiB, 4, 0, 300, False, fail_at)
    assert r["failed"] >= 1
    assert r["completed_cw"] > 0


def test_budget_rejects_oversized_requests(sim):
    r = _run(sim, 4, True, 4 * MiB, 2, 0, 150, True, 5)
    assert r["rejected"] > 0 and r["peak"] <= r["budget"]
