"""Build liblbm_hip.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm_hip.so")
SOURCES = ["lbm_kernels.hip", "lbm_api.hip", "lbm_batch.hip"]
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off: their use is left to nobody
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # contraction only inside one expression: every kernel instance that
    # inlines the node update rounds it identically
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc] + FLAGS + (extra or []) + [os.path.join(CSRC, s) for s in SOURCES] + \
        ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
