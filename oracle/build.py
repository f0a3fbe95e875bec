"""Compile the C oracle (test infrastructure) into oracle/libge_ref.so.

Plain gcc, -O2, no FMA contraction, no fast-math, no explicit SIMD.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libge_ref.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
        "-fno-fast-math", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
        os.path.join(HERE, "ge_ref.c"), os.path.join(HERE, "sdc_ref.c"), "-o", LIB + ".tmp",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
