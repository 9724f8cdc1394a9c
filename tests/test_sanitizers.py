"""The host C/C++ code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the oracle (every entry point, driven by oracle_sanitize.c on
small scans, edge cases included) and the GPU path's geometry compiled for the
host (geometry_host.cpp).  Any out-of-bounds access, leak, signed overflow or
misaligned access aborts the program and fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="4")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="host compilers missing")


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-std=c99", "-D_DEFAULT_SOURCE", "-fopenmp", "-ffp-contract=off", *SAN,
                           os.path.join(HERE, "oracle_sanitize.c"), "-o", exe, "-lm"])
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ok" in r.stdout


@pytest.mark.parametrize("mode", ["ray", "voxel"])
def test_device_geometry_under_sanitizers(tmp_path, mode):
    exe = str(tmp_path / "geometry_san")
    subprocess.check_call(["g++", "-std=c++17", "-ffp-contract=off", "-D__host__=", "-D__device__=",
                           "-D__forceinline__=inline", *SAN, os.path.join(HERE, "geometry_host.cpp"), "-o", exe,
                           "-lm"])
    for N, M, C in ((1, 1, 1), (5, 7, 6), (37, 23, 41), (64, 1, 64), (24, 10, 23), (128, 45, 128)):
        out = str(tmp_path / f"{mode}_{N}.bin")
        r = subprocess.run([exe, mode, str(N), str(M), str(C), out], capture_output=True, text=True, env=ENV,
                           timeout=300)
        assert r.returncode == 0, r.stderr[-4000:]
        assert os.path.getsize(out) > 0
