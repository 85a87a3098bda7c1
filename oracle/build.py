"""Compile the CPU FP64 oracle (plain C99, gcc) into oracle/libhj_oracle.so.

Test infrastructure: the product library never loads this object.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hj_oracle.c")
LIB = os.path.join(HERE, "libhj_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-std=c99", "-Wall", "-Wextra",
        "-ffp-contract=off", "-fno-fast-math",
        "-fopenmp", "-fPIC", "-shared", SRC, "-o", LIB + ".tmp", "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
