"""The library's host code under the sanitizers, on the CPU: argument
checks, table generation, the tuning-table loader fed damaged files and the
serving loop's scheduler (simulate mode, several submitting threads), built
with AddressSanitizer + UndefinedBehaviorSanitizer, and the scheduler again
under ThreadSanitizer. The kernel launchers are stand-ins (no kernel runs)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_11353_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
HOST_UNITS = ["params.cpp", "capi.cpp", "pool.cpp", "tune.cpp", "batch.cpp", "serve.cpp", "he.cpp"]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(tmp_path, name, sanitize, compiler=None):
    gxx = compiler or shutil.which("g++")
    if not gxx or not os.path.exists(gxx) or not os.path.exists(os.path.join(ROCM, "lib", "libamdhip64.so")):
        pytest.skip("the host compiler or the HIP runtime library is not available")
    exe = str(tmp_path / name)
    srcs = [os.path.join(CSRC, u) for u in HOST_UNITS] + [os.path.join(NATIVE, "launch_stubs.cpp"),
                                                         os.path.join(NATIVE, "host_sanitize_test.cpp")]
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", os.path.join(ROCM, "include")] + sanitize + \
        srcs + ["-o", exe, "-L", os.path.join(ROCM, "lib"), "-Wl,-rpath," + os.path.join(ROCM, "lib"),
                "-lamdhip64", "-lrocprofiler-sdk-roctx", "-lpthread", "-ldl"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        if "sanitizer" in r.stderr and ("cannot find" in r.stderr or "not found" in r.stderr):
            pytest.skip("sanitizer runtime not installed")
        raise AssertionError(r.stderr[-4000:])
    return exe


def run(exe, args, env_extra):
    env = dict(os.environ, **env_extra)
    env["NTT_TUNE_CACHE"] = ""          # no table loaded behind the test's back
    out = subprocess.run([exe] + args, capture_output=True, text=True, timeout=600, env=env)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), (out.stdout + out.stderr)[-6000:]


def valid_table(tmp_path):
    """The shipped gfx950 table relabelled with the arch this machine reports
    (the loader refuses other architectures)."""
    import paper_2405_11353_amd as ntt
    f = tmp_path / "arch.json"
    ntt.ntt_tune_clear()
    ntt.ntt_tune_save(str(f))
    arch = f.read_text().split('"arch": "')[1].split('"')[0]
    src = open(os.path.join(ROOT, "paper_2405_11353_amd", "tune_gfx950.json")).read()
    g = tmp_path / "valid.json"
    g.write_text(src.replace('"arch": "gfx950"', '"arch": "%s"' % arch))
    return str(g)


@pytest.mark.slow
def test_host_code_under_asan_and_ubsan(tmp_path):
    exe = build(tmp_path, "host_asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"])
    run(exe, ["all", valid_table(tmp_path), str(tmp_path / "scratch.json")],
        {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1", "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
         "LSAN_OPTIONS": "suppressions=" + os.path.join(NATIVE, "lsan_hip.supp")})


@pytest.mark.slow
def test_server_scheduler_under_tsan(tmp_path):
    # clang's ThreadSanitizer runtime: GCC 11's does not intercept the
    # pthread_cond_clockwait that std::condition_variable::wait_for uses, and
    # then reports the mutex it releases as locked twice
    exe = build(tmp_path, "host_tsan", ["-fsanitize=thread"], os.path.join(ROCM, "llvm", "bin", "clang++"))
    run(exe, ["server"], {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"})
