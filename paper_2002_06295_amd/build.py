"""Build libkfx.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkfx.so")
SOURCES = ["kfx_kernels.hip", "kfx_strips.hip", "kfx_api.hip"]
HEADERS = ["kfx_math.h", "kfx_work.h", "kfx_build.h", "kfx_internal.h"]
ARCH = os.environ.get("KFX_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 (v_pk_*_f32) stays off: hipcc -O3 would form it from
    # plain float code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # contract a*b+c into FMA only within one expression, so that a device
    # function inlined into different kernels rounds identically everywhere
    "-ffp-contract=on",
    # FP32 division and square root by the hardware's reciprocal and square
    # root (within 2.5 ulp) rather than correctly rounded sequences; the FP64
    # parts of the kernels keep correctly rounded division and square root
    "-fno-hip-fp32-correctly-rounded-divide-sqrt",
    # FP32 denormals flushed to zero: the reciprocal and square root then
    # need no range scaling (no FP32 value of these kernels comes near
    # 1e-38; FP64 keeps its denormals)
    "-fgpu-flush-denormals-to-zero",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False, jobs: int = 2) -> str:
    """Compile every source and link the shared library (always rebuilds)."""
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
        if len(procs) >= jobs:
            p, cmd = procs.pop(0)
            if p.wait() != 0:
                raise RuntimeError("compile failed: " + " ".join(cmd))
    for p, cmd in procs:
        if p.wait() != 0:
            raise RuntimeError("compile failed: " + " ".join(cmd))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
