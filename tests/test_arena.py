"""The server's admission arena (hp_arena.h), compiled on its own with the
host compiler and checked against a unit-by-unit occupancy model."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_arena_model(tmp_path):
    exe = tmp_path / "arena_check"
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-I", os.path.join(ROOT, "paper_1505_00914_amd", "csrc"),
                    os.path.join(ROOT, "tests", "arena_check.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert "arena ok" in r.stdout
