"""Build the oracle's shared libraries (test infrastructure only).

``liboracle.so``: ``mbo.c`` compiled with the host C compiler at -O2 without
OpenMP, the checker the tests and the smoke check load.
``liboracle_omp.so``: the same source at -O3 with OpenMP (its pragmas mark
the loops whose iterations are independent), timed by the benchmark's CPU
baseline on the host's cores; it gives the same bits as the checker.
The oracle is a checker for the GPU library; nothing on the product path
links or loads either.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def build(verbose: bool = False, openmp: bool = False) -> str:
    out = LIB_OMP if openmp else LIB
    flags = (["-O3", "-fopenmp", "-Wno-maybe-uninitialized"] if openmp
             else ["-O2", "-Wno-unknown-pragmas"])
    cmd = [
        os.environ.get("CC", "gcc"), *flags,
        "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
        "-o", out + ".tmp", os.path.join(HERE, "mbo.c"), "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build_all(verbose: bool = False):
    return build(verbose), build(verbose, openmp=True)


if __name__ == "__main__":
    build_all(verbose="-v" in sys.argv)
