"""Build the CPU oracle shared library (test infrastructure only).

The oracle is compiled with gcc, single-threaded, with floating-point
contraction and fast-math disabled so that every expression in
resample_oracle.c rounds where it is written. A second build of the same
source with -fopenmp (liboracle_omp.so) serves the all-core CPU baseline; its
parallel loops (Metropolis chains, copied rows) are independent per particle,
so it returns the same bits.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "resample_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-msse2", "-mfpmath=sse", "-Wall", "-Wextra", "-Wno-unused-parameter",
          "-Wno-unknown-pragmas"]


def build(verbose: bool = False, openmp: bool = False) -> str:
    """Compile resample_oracle.c into liboracle.so (or, with openmp, into
    liboracle_omp.so) and return its path."""
    lib = LIB_OMP if openmp else LIB
    tmp = lib + ".tmp"
    cmd = ["gcc", *CFLAGS, *(["-fopenmp"] if openmp else []), SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build_all(verbose: bool = False):
    """Both builds: the single-threaded oracle and the OpenMP baseline."""
    return build(verbose), build(verbose, openmp=True)


if __name__ == "__main__":
    print(*build_all(verbose="-v" in sys.argv))
