"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

libmps.so is rebuilt with the sanitizers on the host pass only (the gfx950
device code is unchanged), a C driver (abi_driver.c) walks every argument
check of the ABI, and the run must finish without a sanitizer report.  Runs
on a host without a GPU (the valid calls end in MPS_ENODEV there).
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2512_20064_amd import build

HERE = os.path.dirname(os.path.abspath(__file__))
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def _gpu_present():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


@pytest.mark.skipif(_gpu_present(), reason="the driver expects the no-device path")
@pytest.mark.skipif(shutil.which(build.hipcc()) is None and not os.path.exists(build.hipcc()), reason="no hipcc")
def test_abi_argument_checks_under_sanitizers(tmp_path):
    cc = build.hipcc()
    inc = os.path.join(build.ROOT, "include")

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        cmd = [cc, "-O1", "-g", "-std=c++17", f"--offload-arch={build.ARCH}", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *SAN,
               "-I", inc, "-x", "hip", "-c", os.path.join(build.CSRC, src), "-o", obj]
        subprocess.run(cmd, check=True, capture_output=True)
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, build.SOURCES))
    lib = str(tmp_path / "libmps_san.so")
    subprocess.run([cc, f"--offload-arch={build.ARCH}", "-shared", "-fPIC", *SAN, *objs, "-o", lib],
                   check=True, capture_output=True)
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_" in syms and "__ubsan_" in syms  # the host code really is instrumented
    exe = str(tmp_path / "abi_driver")
    subprocess.run([cc, *SAN, "-I", inc, "-x", "c", os.path.join(HERE, "abi_driver.c"), "-x", "none", lib,
                    f"-Wl,-rpath,{tmp_path}", "-o", exe], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out
    assert r.returncode == 0 and "ok (0 failures)" in out, out
