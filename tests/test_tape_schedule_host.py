"""The binomial checkpointing schedule of the adjoint's tape (lbm_tape.h),
compiled for the host with g++ (no GPU): a simulated reverse sweep runs
the adjoint steps N-1 .. 0 in order on the right states, within
binom_slots(N) checkpoints, advancing no step more than three times, for
every N up to 400 and a few larger ones."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_binomial_schedule(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "tapechk"
    src = os.path.join(HERE, "native", "tape_schedule_check.cpp")
    subprocess.run([cxx, "-O2", "-std=c++17", "-o", str(exe), src], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "0 failures" in r.stdout
