"""Builds libkfx_hostsim.so: the GPU library's __host__ __device__ math
compiled for the host, for CPU tests of the kernel logic against the oracle.
Test infrastructure only; the library itself never loads it."""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kfx_hostsim.hip")
OUT = os.path.join(HERE, "libkfx_hostsim.so")
CSRC = os.path.join(HERE, "..", "..", "paper_2002_06295_amd", "csrc")


def stale() -> bool:
    if not os.path.exists(OUT):
        return True
    t = os.path.getmtime(OUT)
    deps = [SRC] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    return any(os.path.getmtime(d) > t for d in deps)


def build(force: bool = False) -> str:
    if not force and not stale():
        return OUT
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    cmd = [hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950", "-ffp-contract=on",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", OUT + ".tmp", SRC]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(force=True))
