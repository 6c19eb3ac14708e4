"""The boundary is a C ABI: include/lc.h compiles as C99, and a plain C
program linked against liblc.so (no Python, no torch) runs the five
operations on the GPU and checks them against its own keys."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2412_10770_amd")
ROCM = "/opt/rocm"


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_header_is_c99():
    subprocess.check_call(["gcc", "-x", "c", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                           "-fsyntax-only", os.path.join(ROOT, "include", "lc.h")])


def _build(tmp_path):
    exe = str(tmp_path / "abi_roundtrip")
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-Wall", "-D__HIP_PLATFORM_AMD__",
                           "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "native", "abi_roundtrip.c"),
                           "-L", PKG, "-llc", f"-Wl,-rpath,{PKG}",
                           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-o", exe])
    return exe


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_c_program_links(tmp_path):
    assert os.path.exists(_build(tmp_path))


@pytest.mark.gpu
def test_c_program_roundtrip(tmp_path):
    out = subprocess.run([_build(tmp_path)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "abi roundtrip ok" in out.stdout
