"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and driven through every entry point on small cases by
tests/oracle_asan/asan_driver.c: Cartesian 2D and 3D runs with walls and
periodic axes, plain and deviation storage, both interior-face fluxes, the
single-face fluxes, and the body-fitted 2D and 3D runs.  Any invalid memory
access, leak or undefined operation aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_is_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "orc_asan")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", ORACLE, os.path.join(ROOT, "tests", "oracle_asan", "asan_driver.c"),
           os.path.join(ORACLE, "rtlbfs_oracle.c"), os.path.join(ORACLE, "curv_oracle.c"),
           os.path.join(ORACLE, "curv3_oracle.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "oracle sanitizer run: ok" in r.stdout
