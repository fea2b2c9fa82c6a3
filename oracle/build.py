"""Build the FP64 CPU oracle library (test infrastructure; see lgsr_ref.h).

    python -m oracle.build        # writes oracle/liblgsr_ref.so
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liblgsr_ref.so")


# AddressSanitizer and UndefinedBehaviorSanitizer build of the oracle (CPU only)
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, src: str | None = None, out: str | None = None, sanitize: bool = False) -> str:
    """Compile lgsr_ref.c (or the copy at `src`) into LIB (or `out`); `sanitize` adds the
    address and undefined-behaviour sanitizers."""
    src = src or os.path.join(HERE, "lgsr_ref.c")
    out = out or LIB
    tmp = out + ".tmp"
    # strict IEEE float64: no fast-math, no contraction into FMA
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wextra", *(SANITIZE if sanitize else []), "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
