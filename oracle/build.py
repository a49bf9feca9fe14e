"""Build the FP64 CPU oracle (test infrastructure only) into oracle/liborc.so.

The oracle is compiled with -ffp-contract=off so that every floating-point
operation is rounded on its own; the neighbour inclusion test relies on it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["geometry.cpp", "neighbours.cpp", "potentials.cpp", "cellfilter.cpp", "neb.cpp", "profile.cpp"]
LIB = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
