"""The autotuner's JSON cache (paper_2101_02959_amd/csrc/tune.cpp) is host
C++: build it with the host compiler and run tests/cpp/tune_json_check.cpp
(format round trip, malformed input rejected, cached choices reused)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tune_cache_format(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    src = os.path.join(ROOT, "paper_2101_02959_amd", "csrc")
    exe = tmp_path / "tune_check"
    subprocess.run([cxx, "-std=c++17", "-O1", "-I", src, os.path.join(ROOT, "tests", "cpp", "tune_json_check.cpp"),
                    os.path.join(src, "tune.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("OK")
