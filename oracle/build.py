"""Build the FP64 CPU oracle (test infrastructure, 1D and 2D) into oracle/liboracle.so.

Plain g++ with -O2, no contraction and no fast-math, so that every floating
point operation is the correctly rounded binary64 operation the source names.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wcc_oracle.cpp")       # 1D half-step
SRC2D = os.path.join(HERE, "wcc2d_oracle.cpp")   # 2D half-step
LIB = os.path.join(HERE, "liboracle.so")
# The same sources with OpenMP over the cells of a half-step (identical
# arithmetic; used only to time the oracle on all host cores).
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")

CXXFLAGS = ["-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
            "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    for lib, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        cmd = ["g++", *CXXFLAGS, *extra, "-o", lib + ".tmp", SRC, SRC2D]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(lib + ".tmp", lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
