"""Build the gfx950 HIP library ``librpdla.so`` in-tree with hipcc.

Flags: -O3, C++17, the packed-FP32 feature turned off (float code stays on
the scalar-per-lane VALU path), no fast-math (IEEE infinities and NaNs mark
unborn slots).
"""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "rpdla_api.hip")
HEADERS = [os.path.join(PKG, "csrc", f) for f in
           ("rpdla_device.hpp", "rpdla_kernels.hpp", "rpdla_batched.hpp", "rpdla_fastmath.hpp",
            "rpdla_fastmath_coeffs.hpp", "rpdla_lp_coeffs.hpp")] + \
          [os.path.join(ROOT, "include", "rpdla.h")]
LIB = os.path.join(PKG, "librpdla.so")
ARCH = os.environ.get("RPDLA_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build_library(force: bool = True, verbose: bool = False) -> str:
    """Compile ``csrc/rpdla_api.hip`` (which includes the kernel headers)."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in [SRC] + HEADERS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc] + HIPCC_FLAGS + ["-o", tmp, SRC]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(force=True))
