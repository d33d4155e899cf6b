"""Host-only: the served loop's arena allocator (csrc/server_arena.h), built
with the system C++ compiler and checked by tests/arena_check.cpp (random
allocations from both ends against a bitmap; the serving pattern leaves the
free space in one piece after every batch)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2510_12717_amd", "csrc")


def test_arena_allocator(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "arena_check")
    subprocess.run([cxx, "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "arena_check.cpp"),
                    "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and "arena ok" in out.stdout, out.stdout + out.stderr
