"""Build libntt.so (HIP, gfx950) in-tree with hipcc.

Each kernel translation unit is compiled in its own process (they take tens
of seconds each), then everything is linked into paper_2405_11353_amd/libntt.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libntt.so")
UBENCH = os.path.join(BUILD, "ubench")

ARCH = os.environ.get("NTT_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
# packed-fp32 instructions are disabled for all device code: some of their
# forms have given wrong results on this target without any error
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# NTT_HIPCC_FLAGS: extra flags for tuning builds (e.g. -DNTT_NT_OUT=1)
COMMON = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC] + DEVICE_FLAGS + os.environ.get("NTT_HIPCC_FLAGS", "").split()

KERNEL_UNITS = ["k_u64.hip", "k_u64w.hip", "k_u64x.hip", "k_u32.hip", "k_pointwise.hip", "k_batch.hip", "k_paper.hip", "k_he.hip", "k_polymul.hip",
                "noalloc.hip"]
HOST_UNITS = ["params.cpp", "capi.cpp", "pool.cpp", "tune.cpp", "batch.cpp", "serve.cpp", "he.cpp"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{out}")
    if out.strip():
        print(out, file=sys.stderr)
    return obj


def build(jobs: int = 8, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units = KERNEL_UNITS + HOST_UNITS
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(units)))) as ex:
        objs = list(ex.map(_compile, units))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-lrocprofiler-sdk-roctx"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # the VALU/HBM microbenchmark (a standalone executable)
    cmd = [HIPCC] + COMMON + [os.path.join(CSRC, "ubench.hip"), "-o", UBENCH]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
