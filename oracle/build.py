"""Compile the C part of the oracle into oracle/liboracle.so with gcc.

Test infrastructure: the library never links or loads this.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "imq_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# -ffp-contract=off keeps every entry's rounding exactly as written (no FMA);
# -fno-fast-math keeps IEEE sqrt/divide.
CFLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-std=c11"]


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
