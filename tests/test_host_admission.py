"""Admission policy of the serving runtime, on the CPU (no GPU, no HIP).

tests/admission_sim.cpp drives paper_2309_07270_amd/csrc/xdrop_admission.h --
the pure decision the runtime's submit applies under its lock -- through a
layout that once waited for ever, random submit/complete sequences under
tight HBM budgets (invariants after every step: bytes accounted, budget
kept, a batch that fits alone is admitted whenever no slot is busy, idle
slots released only when that makes room) and producer threads waiting on
one lock and condition variable.  It is built with g++ plain, under
AddressSanitizer + UndefinedBehaviorSanitizer and under ThreadSanitizer.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "admission_sim.cpp")

VARIANTS = {
    "plain": ["-O2"],
    "asan_ubsan": ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"],
    "tsan": ["-O1", "-g", "-fsanitize=thread"],
}


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_admission_policy(tmp_path, variant):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / f"admission_{variant}")
    build = subprocess.run([gxx, "-std=c++17", "-Wall", "-Wextra", "-Werror", "-pthread", *VARIANTS[variant], SRC,
                            "-o", exe], capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "all checks passed" in run.stdout
