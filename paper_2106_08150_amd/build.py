"""Compiles the HIP libraries (gfx950) in-tree.

libmc.so        the classifier (C ABI of include/mc.h)
libmc_peaks.so  memory-system probes used as roofline denominators
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmc.so")
SOURCES = ["mc_api.hip", "mc_build.hip", "mc_query.hip", "mc_server.hip", "mc_condense.hip",
           "mc_noalloc.hip"]
PEAKS_LIB = os.path.join(HERE, "libmc_peaks.so")
PEAKS_SOURCES = ["mc_peaks.hip"]
ARCH = os.environ.get("MC_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed fp32 instructions stay off (none are wanted in integer code)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False) -> str:
    """Compile every source to an object, then link libmc.so (always rebuilds)."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src: str) -> str:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [_hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        if verbose and (r.stdout or r.stderr):
            print(r.stdout, r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES) + len(PEAKS_SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES + PEAKS_SOURCES))
    for lib, n0, n1 in ((LIB, 0, len(SOURCES)), (PEAKS_LIB, len(SOURCES), len(objs))):
        tmp = lib + ".tmp"
        cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs[n0:n1], "-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
