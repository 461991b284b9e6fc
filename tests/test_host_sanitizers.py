"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer:
the HIP sources are compiled with the sanitizers on their host side only
(device code as usual), linked into a driver that exercises the argument
validation of every entry point, the size queries and the host-built mesh
BVH without touching a device, and run in a child process; an invalid
access, overflow or undefined operation aborts it."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2011_03082_amd", "csrc")
SOURCES = ["common", "walk", "cvae", "render", "stats", "mesh"]
CLANG = "/opt/rocm/llvm/bin/clang++"
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="hipcc is needed")
def test_host_code_runs_clean_under_asan_and_ubsan(tmp_path):
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer"]

    def compile_one(name):
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + host_san + [
               "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", os.path.join(CSRC, name + ".hip"),
               "-o", str(tmp_path / (name + ".o"))]
        return subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        for res in ex.map(compile_one, SOURCES):
            assert res.returncode == 0, res.stderr[-3000:]
    drv = str(tmp_path / "host_sanitize.o")
    res = subprocess.run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                          "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-c",
                          os.path.join(ROOT, "tests", "helpers", "host_sanitize.cpp"), "-o", drv],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    exe = str(tmp_path / "host_sanitize")
    objs = [str(tmp_path / (n + ".o")) for n in SOURCES]
    res = subprocess.run([CLANG, "-fsanitize=address,undefined", drv] + objs +
                         ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    # the HIP runtime's own allocations are not this library's: leak checks off
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stderr[-4000:]
    assert "host sanitizer run ok" in run.stdout
