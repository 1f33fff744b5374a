"""Compile the FP64 CPU oracle (test infrastructure) into oracle/_build/liboracle.so.

Plain C99 + OpenMP, no fast-math: the oracle's rounding is IEEE double throughout.
``-fcx-limited-range`` only drops the NaN/Inf recovery of C99 complex multiply,
which finite inputs never reach.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qsv_oracle.c")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liboracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB):
        return LIB
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c99", "-D_GNU_SOURCE", "-O2", "-fopenmp", "-fcx-limited-range",
           "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
