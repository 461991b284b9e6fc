"""Builds the FP64 CPU oracle (plain C, gcc) into oracle/liboracle.so.

Test infrastructure only: the product library never links or loads it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["rng.c", "walk.c", "cvae.c", "render.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
           "-Wno-unused-parameter", "-fno-fast-math", "-ffp-contract=off", "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
