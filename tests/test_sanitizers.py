"""AddressSanitizer + UndefinedBehaviorSanitizer builds (CPU only): the FP64
oracle with a driver that calls every entry point on small ragged inputs, and
the host-only paths of the HIP library (validation, schedule, handles,
SHA-256) with sanitized host code.  Any out-of-bounds access, leak (oracle),
use after free or undefined operation makes the driver exit non-zero."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fopenmp", "-std=c11", "-D_DEFAULT_SOURCE",
                           os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(SAN, "oracle_driver.c"),
                           "-o", exe, "-lm"])
    _run(exe, {"ASAN_OPTIONS": "detect_leaks=1", "OMP_NUM_THREADS": "2"})


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_library_host_paths_under_asan_ubsan(tmp_path):
    import glob
    exe = str(tmp_path / "host_san")
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_1410_0763_amd", "csrc", "*.hip")))
    # sanitizers for the host code only (each -fsanitize= after -Xarch_host)
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include")] + srcs + [os.path.join(SAN, "host_driver.cpp"), "-o", exe]
    subprocess.check_call(cmd)
    _run(exe, {"ASAN_OPTIONS": "detect_leaks=1"})
