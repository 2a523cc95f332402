"""Compiles solve_poisson.c, a plain-C program that calls the C ABI of
libpbcgs.so, with gcc against the HIP runtime.  The program finds the library
through an $ORIGIN-relative rpath, so the tree may move after the build."""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "solve_poisson.c")
EXE = os.path.join(HERE, "solve_poisson")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(out: str = EXE) -> str:
    """Compile the example into `out` (the package's libpbcgs.so must exist)."""
    pkg = os.path.join(ROOT, "paper_1612_01395_amd")
    rel = os.path.relpath(pkg, os.path.dirname(os.path.abspath(out)))
    cmd = ["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-O2", "-D__HIP_PLATFORM_AMD__",
           f"-I{os.path.join(ROOT, 'include')}", f"-I{ROCM}/include", SRC, "-o", out,
           f"-L{pkg}", "-lpbcgs", f"-L{ROCM}/lib", "-lamdhip64", "-lm",
           f"-Wl,-rpath,$ORIGIN/{rel}", f"-Wl,-rpath,{pkg}", f"-Wl,-rpath,{ROCM}/lib"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("gcc failed building the C example")
    return out


if __name__ == "__main__":
    print(build())
