"""Build libsid.so (gfx950) in place with hipcc.

Every source is compiled to its own object (in parallel, under _build/), then
the objects are linked into paper_1905_13257_amd/libsid.so.

Usage: python -m paper_1905_13257_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["csrc/sid_kernels.hip", "csrc/sid_sketch_mfma.hip", "csrc/sid_cpqr.hip",
           "csrc/sid_interp.hip", "csrc/sid_adaptive.hip", "csrc/sid_svd.hip",
           "csrc/sid_apply.hip", "csrc/sid_sketch_f64.hip", "csrc/sid_sketch_v2.hip",
           "csrc/sid_sketch_v2_bf16.hip", "csrc/sid_sketch_v2_bf16x2.hip",
           "csrc/sid_sketch_v2_fp8.hip", "csrc/sid_probe.hip", "csrc/sid_api.hip"]
LIB = os.path.join(HERE, "libsid.so")
OBJDIR = os.path.join(HERE, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _jobs() -> int:
    for var in ("MAX_JOBS", "SID_BUILD_JOBS"):
        v = os.environ.get(var)
        if v and v.isdigit() and int(v) > 0:
            return min(int(v), 16)
    return max(1, min(8, os.cpu_count() or 1))


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = list(SOURCES)
    objs = [os.path.join(OBJDIR, os.path.basename(s).replace(".hip", ".o")) for s in srcs]

    def compile_one(i: int):
        cmd = [hipcc, *HIPCC_FLAGS, "-c", "-o", objs[i], os.path.join(HERE, srcs[i])]
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(compile_one, range(len(srcs))))
    failed = [(s, r) for s, r in zip(srcs, results) if r.returncode != 0]
    if failed:
        for s, r in failed:
            sys.stderr.write(f"---- {s}\n{r.stdout}{r.stderr}")
        raise RuntimeError("hipcc failed building libsid.so: " + ", ".join(s for s, _ in failed))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libsid.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
