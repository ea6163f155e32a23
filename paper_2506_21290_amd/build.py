"""Build script of libflipmc.so (hipcc, gfx950)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "capi.hip", "flex.hip")]
OUT = os.path.join(HERE, "libflipmc.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # contraction only where the code asks for fma(): proposals, wraps and
    # cell indices then round exactly like the FP64 reference definitions
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


# roctx ranges of the host API calls (rocprofv3 --marker-trace)
LINK_FLAGS = ["-lrocprofiler-sdk-roctx"]


def build(verbose: bool = False) -> str:
    cmd = ["hipcc", *HIPCC_FLAGS, "-I" + os.path.join(ROOT, "include"), *SOURCES, "-o", OUT, *LINK_FLAGS]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr[-4000:])
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
