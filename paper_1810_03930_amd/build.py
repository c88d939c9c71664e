"""Build the gfx950 shared library ``libstiefel.so`` in-tree with hipcc.

Usage: ``python -m paper_1810_03930_amd.build`` (or ``build()`` from Python).
The library is written next to this file so that it travels with the source
tree; nothing is installed elsewhere.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB_NAME = "libstiefel.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)
SOURCES = ["stf_kernels.hip", "stf_api.hip", "stf_batched.hip", "stf_adjoint.hip",
           "stf_noalloc.hip"]


def hipcc_path() -> str:
    cand = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(cand):
        raise RuntimeError("hipcc not found; the HIP toolchain is required to build")
    return cand


def build(verbose: bool = True, jobs: int = 4) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    flags = [
        "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
        # no packed-FP32 instructions (v_pk_*_f32) anywhere in the device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-result", "-Wno-unused-value", "-Wno-unused-command-line-argument",
        "-I", os.path.join(HERE, "..", "include"),
    ]
    hipcc = hipcc_path()
    procs = []
    objs = []
    for src in srcs:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [hipcc, *flags, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        while len([p for p in procs if p.poll() is None]) >= jobs:
            procs[0].wait()
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
