"""Build libboltz.so (HIP, gfx950) in-tree with hipcc.

Floating-point contraction is disabled so that every FP64 expression that
decides a node index rounds exactly as written; packed FP32 instructions are
disabled for the device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "boltz.hip")
OUT = os.path.join(HERE, "libboltz.so")
ARCH = os.environ.get("BOLTZ_OFFLOAD_ARCH", "gfx950")


def command(out: str = OUT) -> list[str]:
    return ["hipcc", "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
            "-mcode-object-version=5", "-ffp-contract=off", "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
            SRC, "-o", out]


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
