"""The serving runtime's scheduling policy on a CPU executor (no GPU).

tests/sched_sim.cpp drives paper_2511_09165_amd/csrc/dmas_sched.hpp (the
arena, admission, launch gate and frame grouping that dmas_server.hip uses)
with simulated Poisson arrivals and a simulated device whose streams finish
their launches after varying durations, built with AddressSanitizer and
UndefinedBehaviorSanitizer. It checks, after every step, that granted device
ranges never overlap or leave the budget, that admission follows arrival
order (a frame that does not fit blocks the ones behind it), that every
launch holds one kernel class within the frame and workgroup caps and is led
by the head of the queue, except small launches (at most four device rounds
of workgroups) that start only while the gate is closed and are led by the
first frame that small, and at the end that every admissible frame finished
and the arena coalesced back to one free range.
"""

import json
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sched_sim.cpp")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _build(tmp, extra=()):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = os.path.join(tmp, "sched_sim" + ("_planted" if extra else ""))
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror", *SAN, *extra, "-o", exe, SRC],
                   check=True)
    return exe


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    return _build(str(tmp_path_factory.mktemp("sched")))


def _run(exe, scenario, seed):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, scenario, str(seed)], capture_output=True, text=True, env=env, timeout=120)
    return r


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_mixed_stream(sim, seed):
    r = _run(sim, "mix", seed)
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout)
    assert out["done"] == out["frames"] and out["rejected"] == 0
    assert out["max_used"] <= out["budget"]
    assert out["batched_frames"] > 0 and out["max_group"] > 1            # small frames were packed
    assert out["completed_out_of_launch_order"] >= 1                     # streams finish in any order
    assert out["small_launches"] > 0                                     # small frames went beside long ones


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tight_budget_backpressure(sim, seed):
    r = _run(sim, "tight", seed)
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout)
    assert out["done"] == out["frames"]
    assert out["waits_for_memory"] > 0                                   # admission waited for memory
    assert out["max_used"] <= out["budget"]


def test_frames_beyond_the_budget_are_refused(sim):
    r = _run(sim, "oversize", 5)
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout)
    assert out["rejected"] == len([i for i in range(out["frames"]) if i % 17 == 5])
    assert out["done"] + out["rejected"] == out["frames"]


def test_one_plain_launch_per_frame(sim):
    r = _run(sim, "single", 4)
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout)
    assert out["launches"] == out["frames"] and out["max_group"] == 1 and out["batched_frames"] == 0
    assert out["small_launches"] == 0                                    # one stream: nothing runs beside


def test_checks_catch_a_planted_overtake(tmp_path):
    exe = _build(str(tmp_path), extra=("-DSCHED_SIM_PLANT_OVERTAKE",))
    r = _run(exe, "tight", 1)
    assert r.returncode == 1
    assert "admitted before" in r.stderr
