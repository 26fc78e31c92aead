"""Build step of the package: compiles the HIP kernels and the host runtime
into ``liblge.so`` (gfx950) next to this file, and the input generators."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblge.so")
SOURCES = [os.path.join(CSRC, "lge_kernels.hip"), os.path.join(CSRC, "lge_host.cpp"),
           os.path.join(CSRC, "lge_hostmath.cpp"), os.path.join(CSRC, "lge_server.cpp")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off", "-fvisibility=hidden",
    "-I", os.path.join(ROOT, "include"),
]


def build_lib(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc"] + HIPCC_FLAGS + SOURCES + ["-o", tmp, "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building liblge.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


def build_all() -> None:
    from .inputs import build as build_inputs

    build_inputs(force=True)
    build_lib()


if __name__ == "__main__":
    build_all()
    print(LIB)
