"""Scheduling logic of the tile server, on the CPU: the server's source is built
with g++ against host stand-ins for the HIP runtime and the libfpm calls
(tests/native), then driven through its C ABI."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
SERVER_SRC = os.path.join(ROOT, "paper_2408_13782_amd", "csrc", "fpm_serve.hip")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_server_scheduling_logic(tmp_path):
    exe = tmp_path / "serve_logic"
    cmd = ["g++", "-std=c++17", "-O1", "-pthread", "-I", NATIVE, "-I",
           os.path.join(ROOT, "include"), "-x", "c++", SERVER_SRC, "-x", "none",
           os.path.join(NATIVE, "fake_fpm.cpp"), os.path.join(NATIVE, "serve_logic.cpp"),
           "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip().endswith("OK")
