"""Build libhbc.so (host C++ with g++, device code with hipcc for gfx950)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libhbc.so")
BUILD = os.path.join(ROOT, "_build")

HOST_SOURCES = ["api.cpp", "plan.cpp", "cubed_sphere.cpp", "consumer.cpp"]
DEVICE_SOURCES = ["kernels.hip"]

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
# Packed FP32 instructions are kept out of every device build.
HIP_FLAGS = ["-std=c++17", "-O3", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
CXX_FLAGS = ["-std=c++17", "-O2", "-fPIC", "-Wall", "-Wextra"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for s in HOST_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        jobs.append((o, ["g++", *CXX_FLAGS, "-c", os.path.join(SRC, s), "-o", o]))
    for s in DEVICE_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        jobs.append((o, [HIPCC, *HIP_FLAGS, "-c", os.path.join(SRC, s), "-o", o]))
    with ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(lambda j: _run(j[1]), jobs))
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *[o for o, _ in jobs], "-o", tmp])
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
