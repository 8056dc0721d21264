"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and run over every entry point on small 2D and 3D
problems, edge cases included (oracle/sanitize_driver.c): any out-of-bounds
access, use after free, leak or undefined arithmetic ends the run with an
error."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc on this host")
    exe = str(tmp_path / "oracle_sanitized")
    cmd = [gcc, "-std=c99", "-g", "-O1", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fopenmp",
           "-ffp-contract=off", os.path.join(ROOT, "oracle", "gmres_oracle.c"),
           os.path.join(ROOT, "oracle", "sanitize_driver.c"), "-lm", "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0 and "sanitize" in res.stderr:
        pytest.skip("gcc without the sanitizer runtimes: " + res.stderr[-300:])
    assert res.returncode == 0, res.stderr[-3000:]
    # verify_asan_link_order=0: another preloaded library may come before
    # the sanitizer runtime in the process; the checks themselves are unaffected
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert "oracle sanitizer run: ok" in run.stdout
