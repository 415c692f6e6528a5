"""The library's host code under AddressSanitizer and UBSan (CPU only).

tests/host_sanitize_driver.cpp calls the host-only entry points (rn_version,
rn_strerror, rn_opts_default, rn_validate, rn_footprint and rn_create's
argument check) over valid and invalid problems in host memory. The library's
sources are compiled with the sanitizers on their host code only (the device
code is built as usual and never launched: nothing here reaches a GPU), linked
with ROCm's clang and its sanitizer runtimes, and the driver must exit cleanly
with every status as documented. Leak checking is off: the HIP runtime the
library links keeps allocations until exit.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1908_03301_amd", "csrc")
SOURCES = ["rn_api.cpp", "rn_engine.cpp", "rn_kernels.hip", "rn_fbm.hip", "rn_backbone.hip"]
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.timeout(600)
def test_host_code_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang++"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers are not available")
    objs = []
    for src in SOURCES:
        obj = str(tmp_path / (src + ".o"))
        cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + HOST_SAN + \
              ["-x", "hip", "-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        objs.append(obj)
    drv = str(tmp_path / "drv.o")
    r = subprocess.run([clang, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                        "-I", os.path.join(ROOT, "include"), "-c", os.path.join(HERE, "host_sanitize_driver.cpp"),
                        "-o", drv], capture_output=True, text=True)
    if r.returncode != 0 and "clang_rt" in r.stderr:
        pytest.skip("clang's sanitizer runtimes are not installed")
    assert r.returncode == 0, r.stderr[-2000:]
    exe = str(tmp_path / "host_sanitize_driver")
    r = subprocess.run([clang, "-fsanitize=address,undefined", drv] + objs +
                       ["-o", exe, "-L/opt/rocm/lib", "-lamdhip64", "-lhipfft", "-Wl,-rpath,/opt/rocm/lib"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "verify_asan_link_order=0:detect_leaks=0"
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout + run.stderr[-3000:]
    assert "0 failures" in run.stdout
