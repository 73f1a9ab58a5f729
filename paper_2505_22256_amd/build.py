"""Build the HIP library liblbm.so for gfx950 (in-tree).

hipcc compiles the device code for gfx950 only.  Packed FP32 instructions
are disabled (-packed-fp32-ops); hipcc's host pass warns that it does not
know the feature, which is harmless.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbm.so")
SOURCES = [os.path.join(CSRC, "lbm_api.hip"), os.path.join(CSRC, "lbm_batch.hip")]
HEADERS = [os.path.join(CSRC, n) for n in ("lbm_device.hpp", "lbm_kernels.hpp", "lbm_params.hpp",
                                            "lbm_contact.hpp")] + [os.path.join(ROOT, "include", "lbm.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(force: bool = True, verbose: bool = False) -> str:
    srcs = [s for s in SOURCES if os.path.exists(s)]
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(f) for f in srcs + HEADERS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force=True, verbose=True)
    print(LIB)
    sys.exit(0)
