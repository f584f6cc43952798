"""Build the FP64 CPU oracle (plain C, gcc) into oracle/liboracle.so.

Test infrastructure only.  Floating-point contraction is switched off so
every product and sum is rounded as written.  OpenMP shares the rows of the
lattice update among threads (cells are independent, so results do not
depend on the thread count)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "iblb_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-shared", "-fPIC", "-o", LIB, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
