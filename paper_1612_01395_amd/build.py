"""Builds the HIP library libpbcgs.so for gfx950 in the package directory.

hipcc cross-compiles without a GPU.  Flags: -ffp-contract=off keeps every
+ and * a separately rounded binary64 operation (the library's arithmetic
contract); the device target feature -packed-fp32-ops keeps the compiler from
forming packed binary32 instructions.  hipcc's host pass warns that x86 does
not know that feature; the device pass honours it (tests/test_build_flags.py
shows the difference on a small kernel and checks the built library's device
code for packed binary32 instructions).
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpbcgs.so")
SOURCES = ["pbcgs.hip", "assemble.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("PBCGS_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fvisibility=default",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libpbcgs.so; returns its path."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libpbcgs.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
