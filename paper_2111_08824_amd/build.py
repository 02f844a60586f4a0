"""Build ``liblj.so`` (HIP for gfx950) in-tree with hipcc.

Usage: ``python -m paper_2111_08824_amd.build`` or ``build_lib(force=True)``.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblj.so")

SOURCES = ["lj_build.cpp", "lj_kernels.hip", "lj_partition.hip", "lj_sortjoin.hip", "lj_microbench.hip", "lj_api.cpp", "lj_batch.cpp",
           "lj_server.cpp", "lj_noalloc.cpp"]
HEADERS = ["rmi_eval.h", "lj_internal.h", "lj_device.h", "lj_batch.h", "lj_sortjoin.h", os.path.join("..", "..", "include", "lj.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # The error bounds are only valid if host and device evaluate the models
    # bit-identically: no contraction into fma beyond the explicit ones, no
    # fast-math.
    "-ffp-contract=off",
    "-fno-fast-math",
    # Never emit packed FP32 instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.isabs(c) and os.path.exists(c):
            return c
    return "hipcc"


def _stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, f) for f in SOURCES + HEADERS] + [__file__]
    return any(os.path.getmtime(d) > t for d in deps)


def build_lib(force: bool = False, verbose: bool = False) -> str:
    """Compile every source into liblj.so beside this file."""
    if not force and not _stale():
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include"), "-o", tmp]
    cmd += ["-x", "hip"] + [os.path.join(CSRC, f) for f in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building liblj.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_lib(force=True, verbose=True))
