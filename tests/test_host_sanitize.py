"""The host code that prepares operators (CSR checks and the CSR of A^T,
16-bit column indices, the stored value formats, the matrix-core PSF rows:
csrc/host_ops.hpp, the code the library runs on caller arrays) built with
g++ under AddressSanitizer and UndefinedBehaviorSanitizer and run on random
and malformed inputs, every result checked against a direct computation
(tests/host_ops_check.cpp).  CPU only."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2409_05239_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "host_ops_check.cpp")


def test_host_ops_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the ROCm headers are not installed")
    exe = str(tmp_path / "host_ops_check")
    sanitize = ["-fsanitize=" + s for s in ("address", "undefined")]
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *sanitize,
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           f"-I{CSRC}", SRC, "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "host checks ok" in run.stdout
    assert "runtime error" not in run.stderr
