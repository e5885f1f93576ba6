"""Compile the oracle's C code (oracle/direct.c, oracle/ewald.c) into oracle/_build/liboracle.so with gcc.

Plain -O2 with OpenMP; no fast-math, so the sums follow IEEE FP64 semantics.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD, "liboracle.so")
SOURCES = ("direct.c", "ewald.c")


def build(force: bool = True) -> str:
    srcs = [os.path.join(HERE, f) for f in SOURCES]
    if not force and os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(f) for f in srcs):
        return LIB
    os.makedirs(BUILD, exist_ok=True)
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", *srcs, "-o", tmp, "-lm"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
