"""The decode kernels' digit-group arithmetic on the device table layout
(dtans_core.hpp), compiled for the host and checked against the plain
definition of appending mixed-radix digits (CPU only; the device forms of the
same formulas are covered by the GPU parity tests)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_group_arithmetic_matches_definition(tmp_path):
    exe = str(tmp_path / "core_arith")
    subprocess.run(["g++", "-std=c++17", "-O2", "-I", os.path.join(ROOT, "paper_2603_01915_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "core_arith.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert " 0 failures" in r.stdout
