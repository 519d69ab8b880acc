"""The GPU library's modular arithmetic compiled for the host and checked
against exact 128-bit arithmetic (quotient estimates, lazy-range invariants
of the butterflies, canonicalisation, general products)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "modarith_host_test.cpp")
CSRC = os.path.join(ROOT, "paper_2405_11353_amd", "csrc")


def test_modarith_on_host(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "modarith_host_test")
    # host-only build of the HIP header (-x c++ keeps hipcc from adding device passes)
    subprocess.check_call([hipcc, "-x", "c++", "-O2", "-std=c++17", "-I", CSRC, "-I", "/opt/rocm/include",
                           "-D__HIP_PLATFORM_AMD__",
                           SRC, "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr
