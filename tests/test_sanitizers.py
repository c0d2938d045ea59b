"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the host code (CPU
only): the library's host encoder, container I/O and host decoder
(encoder.cpp), and the oracle's reference codec (dtans_oracle.c), each
driven through encode / write / read / decode round trips of seeded random
and edge-case matrices.  Any memory error or undefined behaviour aborts the
run (-fno-sanitize-recover)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:])
    return r


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_encoder_under_sanitizers(tmp_path):
    exe = str(tmp_path / "enc")
    csrc = os.path.join(ROOT, "paper_2603_01915_amd", "csrc")
    _run(["g++", "-std=c++17"] + SAN + ["-I", csrc, "-I", os.path.join(ROOT, "include"),
          os.path.join(HERE, "encoder_roundtrip.cpp"), os.path.join(csrc, "encoder.cpp"),
          "-o", exe, "-lpthread"], str(tmp_path))
    r = _run([exe, str(tmp_path / "rt.dtans")], str(tmp_path))
    assert " 0 failures" in r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "orc")
    _run(["gcc", "-std=gnu11"] + SAN + [os.path.join(HERE, "oracle_roundtrip.c"),
          os.path.join(ROOT, "oracle", "dtans_oracle.c"), "-fopenmp", "-o", exe], str(tmp_path))
    r = _run([exe, str(tmp_path / "rt.dtans")], str(tmp_path))
    assert " 0 failures" in r.stdout
