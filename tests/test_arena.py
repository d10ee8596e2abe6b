"""The render server's device-memory arena (host logic, no GPU): a randomised
C++ check of allocation, partial release and coalescing."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_arena_blocks_disjoint_and_coalesce(tmp_path):
    exe = tmp_path / "arena_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-o", str(exe),
                    os.path.join(HERE, "native", "arena_check.cpp")], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
