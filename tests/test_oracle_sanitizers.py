"""The oracle under AddressSanitizer and UBSan (CPU only).

tests/oracle_sanitize_driver.c includes oracle/rn_oracle.c as one
translation unit and calls every entry point on small seeded networks (2D and
3D, every flow axis, no-flow and periodic sides, dilution near threshold,
degenerate extents, invalid arguments). Any out-of-bounds access, leak or
undefined behaviour aborts the run.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def test_oracle_under_sanitizers(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc is not available")
    exe = tmp_path / "oracle_sanitize_driver"
    build = subprocess.run([cc] + FLAGS + [os.path.join(HERE, "oracle_sanitize_driver.c"), "-o", str(exe), "-lm"],
                           capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr:
        pytest.skip("the sanitizer runtimes are not installed: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "verify_asan_link_order=0"
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "0 failures" in run.stdout
