"""Builds the HIP library libsgfs.so for gfx950 in-tree (hipcc, no JIT cache).

Usage: python -m paper_1910_11505_amd.build [--verbose]
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsgfs.so")
SOURCES = ["sg_host.cpp", "sg_api.cpp", "sg_kernels.hip", "sg_rapply.hip", "sg_rapply_blocks_64.hip",
           "sg_rapply_blocks_54.hip", "sg_rapply_blocks_63.hip", "sg_rapply_blocks_small.hip",
           "sg_cnn.hip", "sg_mg.hip", "sg_q2.hip"]
ARCH = os.environ.get("SG_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off in every HIP translation unit
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the compile-time index tables of the largest chaos spaces (P = 210)
    "-fconstexpr-steps=50000000",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    t0 = time.time()
    # the translation units compile in parallel (the register-apply unit is the
    # long one)
    jobs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *COMMON, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((src, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.PIPE, text=True)))
    objs, failed = [], []
    for src, obj, proc in jobs:
        out, err = proc.communicate()
        if proc.returncode != 0:
            sys.stderr.write(out + err)
            failed.append(src)
        elif verbose and err.strip():
            sys.stderr.write(err)
        objs.append(obj)
    if failed:
        raise RuntimeError(f"hipcc failed on {', '.join(failed)}")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f} s", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose="--verbose" in sys.argv)
