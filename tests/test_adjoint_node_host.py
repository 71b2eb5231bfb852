"""The per-node hand-written adjoints (lbm_adjoint.h) against central
differences of the per-node forward maps, compiled for the host with g++
(no GPU): dot-product test <l, (f(x+ed)-f(x-ed))/2e> == <adj(l), d>."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_node_adjoints_match_finite_differences(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "adjchk"
    src = os.path.join(HERE, "native", "adjoint_node_check.cpp")
    subprocess.run([cxx, "-O2", "-std=c++17", "-o", str(exe), src], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "0 failures" in r.stdout
