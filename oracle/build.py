"""Build the FP64 CPU oracle (test infrastructure) as a shared library with gcc.

The oracle is plain C compiled without fast-math so that its floating point
follows IEEE semantics; OpenMP only parallelises the loop over independent
(level, sample) pairs.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mlsgd_oracle.c")
LIB = os.path.join(HERE, "libmlsgd_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-Wall", "-Wno-unused-function",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
