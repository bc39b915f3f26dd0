"""Build the HIP library ``libpermest.so`` for gfx950 (cross-compiles
without a GPU).  Run as ``python -m paper_2608_15390_amd.build``."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = [os.path.join(PKG, "csrc", "perm_est.hip")]
HEADERS = [os.path.join(PKG, "csrc", f) for f in ("device.hpp", "traj.hpp", "mlp.hpp", "rows.hpp", "rows_learned.hpp", "prep.hpp", "reduce.hpp", "consensus.hpp")]
LIB = os.path.join(PKG, "libpermest.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no contraction into FMA: the binary32 sums and the FP64 weight
    # arithmetic must round exactly like the sequential definition
    "-ffp-contract=off",
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core results in ordinary VGPRs: the learned trajectory kernel
    # then fits 4 waves per SIMD (AGPRs would round it past 128 registers)
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    "-Wall",
    "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SRC + HEADERS + [os.path.join(ROOT, "include", "perm_est.h")])


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
