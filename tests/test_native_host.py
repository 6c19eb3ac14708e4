"""Host-testable pieces of the native code, compiled with g++ (address and
undefined-behaviour sanitizers on) and run on the CPU: the request server's
output arena (csrc/lc_arena.h) against random alloc/free sequences, the
point queries' searches (csrc/lc_search.h) against linear scans, and the fit
kernels' one-round division (csrc/lc_arith.h) against integer division."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(tmp_path, name, expect):
    exe = str(tmp_path / name)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-fsanitize=address,undefined",
                           "-I", os.path.join(ROOT, "paper_2412_10770_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", name + ".cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert expect in out.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_arena(tmp_path):
    _run(tmp_path, "arena_test", "arena ok")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_searches(tmp_path):
    _run(tmp_path, "search_test", "search ok")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_one_round_division(tmp_path):
    _run(tmp_path, "div_test", "div ok")
