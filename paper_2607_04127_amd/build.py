"""Build the gfx950 renderer library ``liblgsr.so`` in-tree with hipcc.

    python -m paper_2607_04127_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblgsr.so")
SOURCES = ["lgsr_host.hip", "project.hip", "sort.hip", "raster.hip", "loss.hip", "objective.hip", "scan.hip", "chain.hip", "adam.hip", "probe.hip"]
ARCH = os.environ.get("LGSR_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # strict float32: no contraction beyond the explicit fmaf calls, so the forward and the
    # backward evaluate the per-(ray, surfel) test bit-identically
    "-ffp-contract=off",
    # no packed float32 (v_pk_*_f32) code generation
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


# host code only: AddressSanitizer and UndefinedBehaviorSanitizer for the CPU side of the
# library (device code is built as always)
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer"]


def build(verbose: bool = False, extra=None, out: str | None = None, host_sanitize: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out = out or LIB
    tmp = out + ".tmp"
    cmd = [hipcc, *FLAGS, *(HOST_SANITIZE if host_sanitize else []), *(extra or []), "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
