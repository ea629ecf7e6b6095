"""AddressSanitizer / UndefinedBehaviorSanitizer runs of the host code on the CPU.

  * tests/oracle_san.c drives the FP64 oracle (oracle/dmas_oracle.c, built
    from source here with the sanitizers) through every entry point on
    small inputs, edge sizes and invalid arguments;
  * tests/validate_san.cpp drives the plan-description checks that
    dmas_plan_create runs before any device work
    (paper_2511_09165_amd/csrc/dmas_validate.hpp) through every rejection path
    and a seeded fuzz over field values.
The serving scheduler's policy runs under the same sanitizers in
tests/test_sched_sim.py. No GPU is needed.
"""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")


def _run(cmd, exe):
    subprocess.run(cmd, check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok "), r.stdout
    return int(r.stdout.split()[1])


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_san")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-Wall", "-Wextra", "-Werror", "-fopenmp", "-ffp-contract=off", *SAN,
           "-o", exe, os.path.join(HERE, "oracle_san.c"), os.path.join(ROOT, "oracle", "dmas_oracle.c"), "-lm"]
    assert _run(cmd, exe) > 500


def test_plan_description_checks_under_sanitizers(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = str(tmp_path / "validate_san")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror", *SAN, "-I", os.path.join(ROOT, "include"),
           "-o", exe, os.path.join(HERE, "validate_san.cpp")]
    assert _run(cmd, exe) > 20000
