"""Builds the HIP library libdmt.so (gfx950) in place, next to this file.

    python -m paper_2409_17346_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libdmt.so")
SOURCES = [os.path.join(HERE, "csrc", "dmt_host.hip")]
DEPS = SOURCES + [os.path.join(HERE, "csrc", n) for n in ("dmt_kernels.h", "dmt_geom.h", "dmt_frontier.h", "dmt_verify.h", "dmt_codec.h")] + \
    [os.path.join(ROOT, "include", "dmt.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    "-fconstexpr-steps=200000000",
    # exact IEEE arithmetic: the floors use an error-free TwoSum, so no contraction
    "-ffp-contract=off",
    # packed fp32 instructions stay off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = True) -> str:
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", SO + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(SO + ".tmp", SO)
    return SO


def stale() -> bool:
    if not os.path.exists(SO):
        return True
    t = os.path.getmtime(SO)
    return any(os.path.getmtime(p) > t for p in DEPS)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
