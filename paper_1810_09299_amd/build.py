"""Build the HIP library liblbm_axi.so in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "csrc", "lbm_axi.hip"), os.path.join(HERE, "csrc", "lbm_axi_batch.hip")]
LIB = os.path.join(HERE, "liblbm_axi.so")
ARCH = os.environ.get("LBM_AXI_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit multiply-add contraction: every kernel that inlines the node
    # update rounds it identically, so a case's populations do not depend on
    # which kernel (single case, batch, any tile) advanced it
    "-ffp-contract=off",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    tmp = out + ".tmp"
    cmd = ["hipcc", *FLAGS, *[f"-D{d}" for d in defines], *SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
