"""Build the HIP library liblbm.so for gfx950 (in-tree).

hipcc compiles the device code for gfx950 only.  Packed FP32 instructions
are disabled (-packed-fp32-ops); hipcc's host pass warns that it does not
know the feature, which is harmless.  Mixed-precision fused multiply-adds
(-fma-mix-insts, which fold the FP32-to-FP16 store conversion into the last
multiply-add of the collision) are disabled too: the separate multiply-add
and conversion run 2 % faster in the FP16 step kernels, and the results
stay bitwise independent of the tiling.

Every unit is compiled with -ffp-contract=on: a multiply and an add fuse
into one rounding only where they form one source expression, never across
statements.  HIP's default fuses anywhere within a basic block, so the
fusions (and the last bit of FP32 and 16-bit results) depended on how a
kernel instance happened to be shaped: in the 3-D collide pass the instance
with one thread per column fused one multiply-add more than the one with
four, and their FP32 results differed.  Source-defined fusion makes one
step per launch, two fused steps and every tile round identically.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbm.so")
BUILD_DIR = os.path.join(PKG, "_build")
# the longest units first, so that the parallel build ends soonest
SOURCES = [os.path.join(CSRC, n) for n in ("lbm_launch_f32.hip", "lbm_launch_f16.hip", "lbm_launch_bf16.hip",
                                         "lbm_launch_f64.hip", "lbm_batch.hip", "lbm_api.hip",
                                         "lbm3d_launch_f64.hip", "lbm3d_launch_f32.hip", "lbm3d_launch_f16.hip",
                                         "lbm3d_launch_bf16.hip", "lbm3d_api.hip")]
HEADERS = [os.path.join(CSRC, n) for n in ("lbm_device.hpp", "lbm_kernels.hpp", "lbm_params.hpp", "lbm_contact.hpp",
                                            "lbm_launch.hpp", "lbm_launch_impl.hpp", "lbm3d_kernels.hpp",
                                            "lbm3d_contact.hpp", "lbm3d_launch.hpp", "lbm3d_launch_impl.hpp")] + \
    [os.path.join(ROOT, "include", "lbm.h"), os.path.join(ROOT, "include", "lbm3d.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Xclang", "-target-feature", "-Xclang", "-fma-mix-insts", "-ffp-contract=on",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every translation unit (in parallel) and link liblbm.so."""
    srcs = [s for s in SOURCES if os.path.exists(s)]
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(f) for f in srcs + HEADERS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tag = "%d" % os.getpid()
    objs = [os.path.join(BUILD_DIR, os.path.basename(src) + "." + tag + ".o") for src in srcs]
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    procs, pending = [], list(zip(srcs, objs))
    try:
        while pending or procs:
            while pending and len(procs) < jobs:
                src, obj = pending.pop(0)
                cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
                if verbose:
                    print(" ".join(cmd), flush=True)
                procs.append((subprocess.Popen(cmd), src))
            # wait for whichever compile ends first, so a free slot is
            # refilled at once
            while True:
                done = [(p, sname) for p, sname in procs if p.poll() is not None]
                if done:
                    break
                time.sleep(0.2)
            for proc, src in done:
                procs.remove((proc, src))
                if proc.returncode != 0:
                    raise subprocess.CalledProcessError(proc.returncode, src)
        tmp = LIB + ".tmp" + tag
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    finally:
        for p, _ in procs:
            p.kill()
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
    return LIB


if __name__ == "__main__":
    build(force=True, verbose=True)
    print(LIB)
    sys.exit(0)
