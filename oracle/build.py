"""Build the FP64 CPU oracle library (test infrastructure; see lgsr_ref.h).

    python -m oracle.build        # writes oracle/liblgsr_ref.so
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liblgsr_ref.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "lgsr_ref.c")
    tmp = LIB + ".tmp"
    # strict IEEE float64: no fast-math, no contraction into FMA
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
