"""Build the gfx950 library paper_2107_02750_amd/libdg2.so from csrc/ with hipcc.

Packed FP32 instructions are disabled for all device code; nothing else is special.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdg2.so")
ARCH = "gfx950"


def hipcc_flags():
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-Wall"]


def build(verbose: bool = False, extra=None) -> str:
    src = os.path.join(HERE, "csrc", "dg2.hip")
    tmp = LIB + ".tmp"
    cmd = ["/opt/rocm/bin/hipcc"] + hipcc_flags() + list(extra or []) + ["-o", tmp, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
