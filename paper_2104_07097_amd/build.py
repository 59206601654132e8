"""Build libmhar.so (the HIP library behind include/mhar.h) for gfx950, in-tree."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmhar.so")
SOURCES = [os.path.join(HERE, "csrc", "mhar_kernels.hip"), os.path.join(HERE, "csrc", "mhar_resident.hip"),
           os.path.join(HERE, "csrc", "mhar_precond.hip"), os.path.join(HERE, "csrc", "mhar_lane.hip"),
           os.path.join(HERE, "csrc", "mhar_dikin.hip"), os.path.join(HERE, "csrc", "mhar_noalloc.hip"),
           os.path.join(HERE, "csrc", "mhar_api.cpp")]
HEADERS = [os.path.join(HERE, "csrc", "mhar_device.hpp"), os.path.join(HERE, "csrc", "mhar_internal.hpp"),
           os.path.join(ROOT, "include", "mhar.h")]

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-fPIC", "-shared", "-std=c++17", "-Wall",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit contraction: a*b+c rounds twice unless written as fma(), so the
    # exact chord follows the sequential FP64 order of the line-set formula
    "-ffp-contract=off",
]


def build(out: str = LIB, verbose: bool = False) -> str:
    """Compile the library (always recompiles); returns the path."""
    tmp = out + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-o", tmp, *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stdout + res.stderr)
    os.replace(tmp, out)
    return out


def is_stale(out: str = LIB) -> bool:
    if not os.path.exists(out):
        return True
    t = os.path.getmtime(out)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)
