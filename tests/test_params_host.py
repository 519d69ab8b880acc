"""The library's host-side table generators (twiddles with Shoup companions,
the twist tables of the twisted row pass, the row root) checked against their
definitions with plain 128-bit arithmetic, compiled for the CPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "params_host_test.cpp")
CSRC = os.path.join(ROOT, "paper_2405_11353_amd", "csrc")


def test_tables_match_definitions(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "params_host_test")
    subprocess.check_call([gxx, "-O2", "-std=c++17", "-I", CSRC, SRC, os.path.join(CSRC, "params.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr
    print(out.stdout)
