"""Build libsid.so (gfx950) in place with hipcc.

Usage: python -m paper_1905_13257_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["csrc/sid_kernels.hip", "csrc/sid_sketch_mfma.hip", "csrc/sid_cpqr.hip",
           "csrc/sid_interp.hip", "csrc/sid_adaptive.hip", "csrc/sid_svd.hip",
           "csrc/sid_apply.hip", "csrc/sid_sketch_f64.hip", "csrc/sid_api.hip"]
LIB = os.path.join(HERE, "libsid.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    # rocBLAS for the plain N-length GEMMs of SBR-SVD
    cmd = [hipcc, *HIPCC_FLAGS, "-o", tmp, *srcs, "-L/opt/rocm/lib", "-lrocblas"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libsid.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
