"""Host logic of the request server: its output arena (csrc/lc_arena.h),
compiled with g++ (address and undefined-behaviour sanitizers on) and run
against random alloc/free sequences on the CPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_arena(tmp_path):
    exe = str(tmp_path / "arena_test")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-fsanitize=address,undefined",
                           "-I", os.path.join(ROOT, "paper_2412_10770_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", "arena_test.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert "arena ok" in out.stdout
