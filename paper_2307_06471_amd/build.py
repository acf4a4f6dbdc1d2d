"""Build the HIP library libcrkdg.so for gfx950 in-tree.

hipcc cross-compiles without a GPU.  Flags:
  -ffp-contract=on   fuse a*b+c only inside one source expression, so two
                     copies of the same trace/flux code round identically
                     (face fluxes computed by two tiles stay bit-identical);
  -Xclang -target-feature -Xclang -packed-fp32-ops
                     no packed FP32 instructions.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libcrkdg.so")
SOURCES = ["crkdg_kernels.hip", "crkdg_mlp.hip", "crkdg_api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=on", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def build(verbose: bool = False, extra=None) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    cmd = [HIPCC] + FLAGS + (extra or []) + [os.path.join(SRC, s) for s in SOURCES] + \
        ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
