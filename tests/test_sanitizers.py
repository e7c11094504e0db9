"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the CPU code,
run on the CPU: the FP64 oracle (g++) and the host build of the GPU
library's device math (tests/hostsim, hipcc with the sanitizers on the host
side only), each driven by tests/sanitize/exercise.py in a subprocess with
the sanitizer runtime preloaded.  Any report, or an abort from one (no
recovery), fails the test."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
EXERCISE = os.path.join(HERE, "sanitize", "exercise.py")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def run(cmd_env, args, tmp_path):
    env = dict(os.environ)
    env.update(cmd_env)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    p = subprocess.run([sys.executable, EXERCISE] + args, env=env, cwd=str(tmp_path), capture_output=True,
                       text=True, timeout=900)
    text = p.stdout + p.stderr
    assert p.returncode == 0, text[-4000:]
    assert "AddressSanitizer" not in text and "runtime error" not in text, text[-4000:]
    return text


def test_oracle_under_asan_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    asan = subprocess.run([gxx, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan not available")
    lib = str(tmp_path / "libkfo_san.so")
    subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-shared", "-fPIC", *SAN, "-o", lib,
                    os.path.join(ROOT, "oracle", "kfo.cpp")], check=True)
    out = run({"LD_PRELOAD": asan, "KFO_LIB": lib}, [], tmp_path)
    assert "oracle ok" in out


def test_hostsim_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    rts = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rts:
        pytest.skip("clang ASan runtime not available")
    lib = str(tmp_path / "libhs_san.so")
    host = []
    for f in SAN + ["-shared-libsan"]:
        host += ["-Xarch_host", f]
    subprocess.run([hipcc, "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                    "-ffp-contract=on", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host, "-o", lib,
                    os.path.join(HERE, "hostsim", "kfx_hostsim.hip")], check=True, capture_output=True)
    out = run({"LD_PRELOAD": rts[-1]}, ["--hostsim", lib], tmp_path)
    assert "hostsim ok" in out
