"""Build the HIP library ``liblcs_hip.so`` for gfx950, in-tree.

Plain ``hipcc`` (no torch extension machinery): the library exposes only the
C ABI of ``include/lcs.h`` and links nothing but the HIP runtime.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblcs_hip.so")
ARCH = "gfx950"

SOURCES = ["api.hip", "api_mlp.hip", "api_mesh.hip", "advect.hip", "cgftle.hip", "mlp.hip",
           "mesh.hip", "train.hip"]

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # packed FP32 (v_pk_*_f32) code generation stays off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # contraction to FMA is allowed, except where a function opts out with
    # "#pragma clang fp contract(off)"
    "-ffp-contract=fast-honor-pragmas",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + ["-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
