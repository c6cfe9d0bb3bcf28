"""Compile the FP64 reference oracle (plain C) into oracle/libdem_oracle.so.

The oracle is test infrastructure: it is built beside the product so the
tests, the smoke check and the benchmark's CPU-baseline leg can load it, and
nothing in the product path links it.  Built with -O2 -ffp-contract=off so
that no multiply-add is fused and every expression rounds as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libdem_oracle.so")
SRC = os.path.join(HERE, "dem_oracle.c")
FLAGS = ["-std=c99", "-D_DEFAULT_SOURCE", "-O2", "-ffp-contract=off", "-fno-fast-math",
         "-Wall", "-Wextra", "-fPIC", "-shared"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *FLAGS, "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
