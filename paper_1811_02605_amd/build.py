"""Build step for the HIP library (gfx950).

    python -m paper_1811_02605_amd.build

compiles ``csrc/*.hip`` with hipcc into ``paper_1811_02605_amd/lib/libmas_hip.so``
(in-tree, so it travels with the source tree).
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libmas_hip.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["mas_api.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


C_PROGRAM_SRC = os.path.join(ROOT, "tests", "c_api_solve.c")
C_PROGRAM = os.path.join(LIBDIR, "libc_api_solve.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build_c_program(verbose: bool = False) -> str:
    """The C99 code that solves through include/mas.h with no Python in
    between (a GPU test calls its c_api_solve_run), as a shared library linked
    against the library beside it."""
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-fPIC", "-shared",
           "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), C_PROGRAM_SRC,
           "-L", LIBDIR, "-lmas_hip", "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", C_PROGRAM]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return C_PROGRAM


def build_library(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"),
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
    print(build_c_program(verbose="-v" in sys.argv))
