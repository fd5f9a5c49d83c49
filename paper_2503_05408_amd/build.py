"""Builds ``libgltrsv.so`` (HIP for gfx950 + host C++) in the package folder.

Flags that matter for the results:
  -ffp-contract=off   every binary64 multiply and subtract is rounded on its
                      own, as the solve's operation order requires;
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      no packed FP32 instructions in device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgltrsv.so")
SOURCES_HOST = ["analysis.cpp", "local.cpp", "wave.cpp"]
SOURCES_HIP = ["kernels.hip", "gltrsv.hip", "serve.hip", "pack.hip", "local.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("GLTRSV_ARCH", "gfx950")


def sources():
    return [os.path.join(CSRC, f) for f in SOURCES_HOST + SOURCES_HIP + ["analysis.h", "internal.h", "local.h", "wave.h"]] + [
        os.path.join(ROOT, "include", "gltrsv.h")]


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in sources())


def build(verbose: bool = False, out: str | None = None, defines=()) -> str:
    """Compiles the library to ``out`` (default: the in-package path)."""
    out = out or LIB
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    common = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-I", os.path.join(ROOT, "include")]
    for src in SOURCES_HOST:
        obj = os.path.join(bdir, src + ".o")
        cmd = ["g++", *common, "-Wall", *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", *common,
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           *[f"-D{d}" for d in defines],
           "-shared", *[os.path.join(CSRC, s) for s in SOURCES_HIP], "-x", "none", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
