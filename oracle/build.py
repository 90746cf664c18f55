"""Build the FP64 CPU oracle (test infrastructure) into oracle/liblbimb_oracle.so.

The oracle is compiled with gcc, strict IEEE binary64 semantics: no fast-math,
no floating-point contraction, so every expression rounds exactly as written.
OpenMP splits its per-node and per-particle loops over threads without
changing any result (orc_set_threads(1) gives the serial program).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbimb_oracle.c")
LIB = os.path.join(HERE, "liblbimb_oracle.so")

CFLAGS = ["-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off",
          "-fno-math-errno", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(verbose=False):
    cmd = ["gcc", *CFLAGS, "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
