"""Build the oracle's shared library (test infrastructure only).

Compiles ``mbo.c`` with the host C compiler into ``liboracle.so`` next to it.
The oracle is a checker for the GPU library; nothing on the product path
links or loads it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        os.environ.get("CC", "gcc"),
        "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
        "-o", LIB + ".tmp", os.path.join(HERE, "mbo.c"), "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
