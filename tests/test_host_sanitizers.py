"""The library's host code under host sanitizers: the C-ABI sources built
with AddressSanitizer and UndefinedBehaviorSanitizer on the host side only
(device code is compiled as usual and never run here), linked with a small
driver (tests/host_sanitize_driver.cpp) that runs the host-only entry points:
the hierarchy builders and checks on random, identical and collinear triangle
sets, the information word, the store size, and pv_create's error return
without a GPU.  No GPU."""
import glob
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = "/opt/rocm/bin/hipcc"


def test_host_code_clean_under_asan_and_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2111_06906_amd", "csrc", "*.hip")))
    exe = str(tmp_path / "host_sanitized")
    cmd = [HIPCC, "-std=c++17", "-O1", "-g", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), "-o", exe, os.path.join(HERE, "host_sanitize_driver.cpp")] + srcs
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "sanitized host run done" in r.stdout
