"""Compile the CPU oracle (plain C, FP64, OpenMP) into oracle/liboracle.so.

Test infrastructure only.  -ffp-contract=off keeps every product and sum
an individually rounded IEEE operation, exactly as written in the C source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["graph.c", "irls.c", "sweep.c", "maxflow.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wno-unused-result", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, f) for f in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
