"""Build the HIP library liblc.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblc.so")
SOURCES = [os.path.join(CSRC, "lc_kernels.hip"), os.path.join(CSRC, "lc_api.cpp"), os.path.join(CSRC, "lc_serve.cpp"),
           os.path.join(CSRC, "lc_noalloc.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-fvisibility=hidden",
    "-Wall", "-Wno-unused-function",
    # keep packed fp32 instructions out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(out: str = LIB, extra: list | None = None) -> str:
    tmp = out + ".tmp"
    srcs = [x for src in SOURCES for x in ("-x", "hip", src)]
    cmd = [HIPCC, *FLAGS, *(extra or []), *srcs, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
