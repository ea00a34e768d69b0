"""Build the HIP library libtrbt.so in-tree for gfx950.

    python -m paper_2002_10991_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SRCS = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
OUT = os.path.join(HERE, "libtrbt.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-variable",
]


# Debug variant: every wait between waves is preceded by a pseudo-random
# delay (TRBT_WAIT_JITTER in trbt_device.h), to run the hand-offs in many
# orders.  Loaded instead of the release library with TRBT_LIB=<path>.
OUT_JITTER = os.path.join(HERE, "libtrbt_jitter.so")


def build(verbose: bool = False, out: str = OUT, extra=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + f".tmp{os.getpid()}"
    cmd = [hipcc, *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *SRCS,
           "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build_jitter(verbose: bool = False) -> str:
    return build(verbose, OUT_JITTER, ("-DTRBT_WAIT_JITTER",))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    if "--jitter" in sys.argv:
        print(build_jitter(verbose="-v" in sys.argv))
