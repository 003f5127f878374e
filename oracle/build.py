"""Build the FP64 CPU oracle (test infrastructure) as a shared library.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
the result.  Plain gcc, OpenMP over the output frequencies.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bz_oracle.c")
LIB = os.path.join(HERE, "libbz_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
