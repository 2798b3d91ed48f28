"""Build the CPU oracle (plain C, gcc) into oracle/liboracle.so.

Test infrastructure: compiles only oracle.c, with -ffp-contract=off so that
no multiply-add is fused, and OpenMP for the independent base-index loops.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True, src: str = SRC, out: str = LIB, extra=()) -> str:
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", out + ".tmp", src, "-lm", *extra]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(force=True))
    sys.exit(0)
