"""Build libdem_hip.so (hand-written HIP for gfx950) with hipcc.

    python -m paper_2301_00611_amd.build        # or: python paper_2301_00611_amd/build.py

Every source in csrc/ is compiled to an object in _build/ (in parallel), then
linked into paper_2301_00611_amd/libdem_hip.so.  Device code is compiled with
FMA contraction that honours `#pragma clang fp contract(off)` (the exact
contact test uses it) and with packed-FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libdem_hip.so")
ARCH = os.environ.get("DEM_OFFLOAD_ARCH", "gfx950")

DEVICE_SOURCES = ["prim.hip", "broadphase.hip", "contact.hip", "integrate.hip", "stress.hip"]
HOST_SOURCES = ["runtime.cpp"]

COMMON = ["-std=c++17", "-O3", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall",
          "-Wno-unused-function"]
DEVICE_FLAGS = [f"--offload-arch={ARCH}", "-ffp-contract=fast-honor-pragmas",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-ffp-contract=off", "-D__HIP_PLATFORM_AMD__"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, verbose: bool) -> str:
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [hipcc(), "-x", "hip", *COMMON, *DEVICE_FLAGS, "-c", path, "-o", obj]
    else:
        cmd = [hipcc(), *COMMON, *HOST_FLAGS, "-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip() and verbose:
        print(r.stderr, file=sys.stderr)
    return obj


def build(verbose: bool = False) -> str:
    srcs = DEVICE_SOURCES + HOST_SOURCES
    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), 8)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
