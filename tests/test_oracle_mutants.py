"""The learned-step pins catch the mistakes they are meant to catch: each
case plants one plausible error in a copy of the oracle's C source (an
alpha / beta swap or a sign flip in the exit frame of Sec. 4.1, the wrong
sense of the azimuth psi, a first-event probability off by one term of
Lambda^(N), a single scatter drawn with -g), builds that copy with gcc and
runs the pin against it in a child process, which must fail; the unchanged
copy must pass the same pins."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")

W0 = "double w0[3] = {be * ct + ga * st, al, -be * st + ga * ct};"
PSI = "double cp = cos(psi), sp = sin(psi);"
PFIRST = "double p_first = phi >= 1.0 ? 1.0 / N : (1.0 - phi) / (-expm1(N * log(phi)));"
HG1 = "ct = or_hg_sample(g, u[2]);"

ROUND_TRIP = "T.test_step_reproduces_training_walk_records(oracle)"
FIRST_LAW = "T.test_first_event_law(oracle, 5, 1.0); T.test_first_event_law(oracle, 5, 0.9)"
SINGLE = "T.test_single_event_step_is_one_hg_scatter(oracle, 0.8)"

MUTANTS = {
    "alpha-beta swap": (W0, "double w0[3] = {al * ct + ga * st, be, -al * st + ga * ct};", ROUND_TRIP),
    "beta sign": (W0, "double w0[3] = {-be * ct + ga * st, al, be * st + ga * ct};", ROUND_TRIP),
    "psi sense": (PSI, "double cp = cos(psi), sp = -sin(psi);", ROUND_TRIP),
    "first-event law": (PFIRST, "double p_first = phi >= 1.0 ? 1.0 / (N + 1.0) : "
                                "(1.0 - phi) / (-expm1((N + 1.0) * log(phi)));", FIRST_LAW),
    "single scatter g sign": (HG1, "ct = or_hg_sample(-g, u[2]);", SINGLE),
}


def oracle_copy(tmp_path, find=None, replace=None):
    dst = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), dst,
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    if find is not None:
        src = (dst / "render.c").read_text()
        assert src.count(find) == 1, find
        (dst / "render.c").write_text(src.replace(find, replace))
    return str(tmp_path)


def run_pins(pkg_parent, calls):
    # the copy's parent goes first on the path, so `import oracle` takes the copy
    script = (f"import sys; sys.path[:0] = [{pkg_parent!r}, {TESTS!r}, {ROOT!r}]; import oracle; "
              f"assert oracle.__file__.startswith({pkg_parent!r}), oracle.__file__; "
              f"import test_oracle_step as T; print('copy loaded', flush=True); {calls}")
    return subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, timeout=600)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is needed")
def test_unchanged_copy_passes_the_pins(tmp_path):
    res = run_pins(oracle_copy(tmp_path), "; ".join([ROUND_TRIP, FIRST_LAW, SINGLE]))
    assert res.returncode == 0, res.stderr[-3000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is needed")
@pytest.mark.parametrize("name", list(MUTANTS))
def test_planted_mistake_fails_its_pin(tmp_path, name):
    find, replace, calls = MUTANTS[name]
    res = run_pins(oracle_copy(tmp_path, find, replace), calls)
    assert "copy loaded" in res.stdout, res.stderr[-3000:]
    assert res.returncode != 0, f"{name}: the pin did not notice"
    assert "AssertionError" in res.stderr, res.stderr[-3000:]
