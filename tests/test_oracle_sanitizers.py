"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
every entry point (walks in both modes with focus data, features, CVAE
initialisation / loss and gradient / AdamW / activation scales / sampling in
FP64, BF16 and FP8 for one- and two-tile shapes, plain, exact-walk and
learned renders with and without a distance grid, a mesh) on small inputs,
built with gcc and run in a child process; any invalid access, leak,
overflow or undefined operation aborts it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is needed")
def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    srcs = [os.path.join(ORACLE, f) for f in ("rng.c", "walk.c", "cvae.c", "render.c")]
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", ORACLE, "-o", exe,
           os.path.join(ROOT, "tests", "helpers", "oracle_sanitize.c")] + srcs + ["-lm", "-lpthread"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, run.stderr[-4000:]
    assert "oracle sanitizer run ok" in run.stdout
