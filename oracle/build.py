"""Build the FP64 CPU oracle (test infrastructure) into oracle/libdg2ref.so.

Plain gcc, OpenMP over rows, -ffp-contract=off so expressions round as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libdg2ref.so")


TALLY_LIB = os.path.join(HERE, "libdg2ref_tally.so")


def build(verbose: bool = False) -> str:
    """Builds the oracle and its operation-tally build; returns the oracle's path."""
    src = os.path.join(HERE, "dg2ref.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O3", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    # the same source as C++ with every double a counting Real (oracle/tally.hpp), one
    # thread; -fpermissive lets C's implicit void* conversions of malloc through, and -w
    # keeps it from reporting each of them
    tmp = TALLY_LIB + ".tmp"
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-fpermissive",
           "-w", "-x", "c++", "-include", os.path.join(HERE, "tally.hpp"), "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, TALLY_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
