"""Build the CPU oracle (test infrastructure only) into oracle/liboracle.so.

Plain C, FP64, serial; -ffp-contract=off so that no fused multiply-add
changes the rounding of the reference arithmetic, and never -ffast-math.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "crkdg_oracle.c")
    cmd = ["gcc", "-std=gnu11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-shared", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
