"""Builds libmatexpre.so (HIP for gfx950) in the package directory.

Run as `python paper_2506_03617_amd/build.py` or through __graft_entry__.build()
(not through the package, whose import loads the library being rebuilt).
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmatexpre.so")

SOURCES = ["kernels.hip", "cheb2d.hip", "cheb3d.hip", "cnn.hip", "schedule.cpp", "action.cpp", "krylov.cpp",
           "batch.cpp", "api.cpp", "network.cpp", "checkpoint.cpp", "tunecache.cpp",
           "noalloc.cpp"]

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions are kept out of generated code on purpose
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def build(verbose: bool = False) -> str:
    cc = hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        lang = [] if src.endswith(".hip") else ["-x", "hip"]
        cmds.append([cc, *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), *lang, "-c",
                     os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # the translation units compile independently
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
        for fut in [pool.submit(subprocess.run, cmd, check=True) for cmd in cmds]:
            fut.result()
    tmp = LIB + ".tmp"
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    # roctx ranges around the solver's phases (rocprofv3 --marker-trace)
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-L", os.path.join(rocm, "lib"),
           "-lrocprofiler-sdk-roctx", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
