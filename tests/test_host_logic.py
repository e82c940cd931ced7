"""Host-side bookkeeping of the library, checked on the CPU.

The two-pass workspace registry (one buffer per device and stream, grown but
never freed while the library is loaded, no allocation under capture) is
compiled with g++ against a fake allocator and run.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2412_05824_amd", "csrc")


def _build_and_run(src, tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC,
                    os.path.join(HERE, "host", src), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    return r


def test_workspace_pool_keeps_captured_buffers(tmp_path):
    r = _build_and_run("ws_pool_check.cpp", tmp_path)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().startswith("ok")
