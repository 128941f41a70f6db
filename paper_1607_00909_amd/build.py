"""Build the HIP library in-tree: paper_1607_00909_amd/libcdmt.so for gfx950.

Usage: python -m paper_1607_00909_amd.build   (or __graft_entry__.build())
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", f)
        for f in ("cdmt.hip", "redigit.hip", "incoherent.hip", "plan.cpp")]
DEPS = [*SRCS, os.path.join(HERE, "csrc", "fft_core.hpp"), os.path.join(HERE, "csrc", "plan.hpp"),
        os.path.join(HERE, "csrc", "xcd.hpp"),
        os.path.join(ROOT, "include", "cdmt.h")]
LIB = os.path.join(HERE, "libcdmt.so")
ARCH = os.environ.get("CDMT_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions (v_pk_*_f32) in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def build(verbose: bool = False, save_temps: str | None = None) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), *SRCS, "-o", tmp]
    if save_temps:
        cmd.insert(1, f"-save-temps={save_temps}")
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
