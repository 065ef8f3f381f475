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
# The same sources with OpenMP: the sweep's rows split over threads (used to
# time the oracle on every core; one thread reproduces LIB's arithmetic).
LIB_OMP = os.path.join(HERE, "libdrot_ref_omp.so")


def build(verbose: bool = False) -> str:
    for lib, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-Wall", "-Wextra", *extra, "-o", lib + ".tmp", *SRCS, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(lib + ".tmp", lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
