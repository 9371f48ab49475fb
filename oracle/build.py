"""Build the FP64 CPU oracle (test infrastructure) into oracle/libdg2ref.so.

Plain gcc, OpenMP over rows, -ffp-contract=off so expressions round as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libdg2ref.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "dg2ref.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O3", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
