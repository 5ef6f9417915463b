"""Compile the plain C oracle into oracle/librtlbfs_oracle.so with gcc.

Test infrastructure: the oracle is a checker for the GPU library and is never
part of the product path.  Built without fast-math and without floating-point
contraction so its arithmetic is exactly the order written in the source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rtlbfs_oracle.c")
SRCS = [SRC, os.path.join(HERE, "curv_oracle.c"), os.path.join(HERE, "curv3_oracle.c")]
LIB = os.path.join(HERE, "librtlbfs_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", *SRCS, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
