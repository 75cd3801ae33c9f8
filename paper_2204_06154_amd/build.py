"""Build libmgm.so in-tree: host setup (g++, no FP contraction) + HIP for gfx950.

Usage: python -m paper_2204_06154_amd.build   (or call build())
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmgm.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST_SOURCES = ["knn.cpp", "weights.cpp", "wse.cpp", "hierarchy.cpp"]
HIP_SOURCES = ["device.hip", "phs_batched.hip", "learned.hip", "setup_device.hip", "surface_ops.hip"]
EXACT_HIP_SOURCES = {"setup_device.hip"}


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def _stale(obj: str, src: str) -> bool:
    """True when obj is older than its source or any header of csrc/ or include/."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    deps.append(os.path.join(ROOT, "include", "mgm.h"))
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = True, incremental: bool = False) -> str:
    """Compile every source (incremental=True: only those whose object is
    older than the source or a header) and link libmgm.so."""
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        objs.append(obj)
        if incremental and not _stale(obj, src):
            continue
        _run(["g++", "-std=c++17", "-O2", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-pthread",
              "-Wall", "-c", os.path.join(CSRC, src), "-o", obj])
    for src in HIP_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        objs.append(obj)
        if incremental and not _stale(obj, src):
            continue
        # the device preprocessing must round exactly as the host path does
        contract = "-ffp-contract=off" if src in EXACT_HIP_SOURCES else "-ffp-contract=fast"
        _run([hipcc, "-std=c++17", "-O3", "-fPIC", "--offload-arch=gfx950",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              contract,
              "-c", os.path.join(CSRC, src), "-o", obj])
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-pthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv)
    sys.exit(0)
