"""Compile libspd.so (HIP, gfx950) in-tree."""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libspd.so")
SOURCES = [os.path.join(PKG, "csrc", f) for f in ("spd_kernels.hip", "spd_runtime.hip")]
HEADERS = [os.path.join(ROOT, "include", "spd.h"), os.path.join(PKG, "csrc", "spd_internal.h")]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build_library(verbose: bool = False) -> str:
    """Compile every source for gfx950 into a temporary file, then move it into place."""
    fd, tmp = tempfile.mkstemp(suffix=".so", dir=PKG)
    os.close(fd)
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
           # keep the compiler from emitting packed FP32 instructions
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-o", tmp] + SOURCES
    try:
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("libspd build failed:\n" + res.stderr)
        if verbose:
            print(" ".join(cmd))
        os.replace(tmp, LIB)
    finally:
        if os.path.exists(tmp):
            os.unlink(tmp)
    return LIB


CEIL_LIB = os.path.join(PKG, "libspd_ceilings.so")
CEIL_SOURCES = [os.path.join(PKG, "csrc", "spd_ceilings.hip")]


def build_ceilings(verbose: bool = False) -> str:
    """The microbenchmarks of the hardware ceilings (a library of their own)."""
    fd, tmp = tempfile.mkstemp(suffix=".so", dir=PKG)
    os.close(fd)
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-o", tmp] + CEIL_SOURCES
    try:
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("libspd_ceilings build failed:\n" + res.stderr)
        if verbose:
            print(" ".join(cmd))
        os.replace(tmp, CEIL_LIB)
    finally:
        if os.path.exists(tmp):
            os.unlink(tmp)
    return CEIL_LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build_library(verbose=True))
