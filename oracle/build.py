"""Builds the oracle's shared library (liboracle.so) with the host C compiler.

Test infrastructure: the library is loaded only by the test suite, the smoke
check and the benchmark's CPU-baseline leg.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pms_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O3", "-march=x86-64-v2", "-std=c11", "-fPIC", "-shared", "-pthread",
          "-Wall", "-Wextra"]


def build(src: str = SRC, out: str = LIB, extra=()) -> str:
    """Compiles ``src`` into the shared library ``out`` and returns its path."""
    cc = os.environ.get("CC", "gcc")
    tmp = out + ".tmp"
    cmd = [cc, *CFLAGS, *extra, src, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(*sys.argv[1:2]))
