"""The oracle and the library's host-only planning code built with
AddressSanitizer and UndefinedBehaviorSanitizer (host code only), driven over
small inputs and a range of volumes, partitions and views
(``tests/sanitize/*_driver.*``): the drivers must exit cleanly with no
sanitizer report."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

pytestmark = pytest.mark.slow


def _run(exe, tmp_path):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, cwd=str(tmp_path), timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fopenmp", "-std=c11",
                           os.path.join(HERE, "sanitize", "oracle_driver.c"), os.path.join(ROOT, "oracle", "vr_oracle.c"),
                           "-o", exe, "-lm"])
    assert "oracle driver: ok" in _run(exe, tmp_path)


def test_planning_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_driver")
    csrc = os.path.join(ROOT, "paper_1008_0135_amd", "csrc")
    # host code only: the sanitizers apply to the host compilation
    subprocess.check_call([HIPCC, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-I", os.path.join(ROOT, "include"), "-I", csrc,
                           os.path.join(HERE, "sanitize", "plan_driver.cpp"), os.path.join(csrc, "plan.cpp"),
                           "-o", exe], stderr=subprocess.DEVNULL)
    assert "plan driver: 0 failed checks" in _run(exe, tmp_path)
