"""Build the oracle's C library (oracle/libdrot_ref.so: the FP64 DROT of
drot_ref.c and the network simplex of netsimplex.c) with gcc.

Test infrastructure: compiled by the package build step so that the tests
and the CPU-baseline leg of the benchmark find it; nothing in the GPU path
links or loads it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "drot_ref.c"), os.path.join(HERE, "netsimplex.c")]
LIB = os.path.join(HERE, "libdrot_ref.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", *SRCS, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
