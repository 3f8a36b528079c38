"""Builds libhenn.so (HIP, gfx950) in-tree with hipcc.

Each .hip source is compiled separately, then linked into one shared library
next to this file.  Packed FP32 instructions are switched off for the device
code (-packed-fp32-ops): the kernels are written in scalar FP32.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhenn.so")
# (source, object, extra flags): henn_search.hip builds in four parts (host
# functions and root kernels; the FP32 / BF16 / FP8 search kernels)
SOURCES = [("henn_api.hip", "henn_api", []),
           *[("henn_search.hip", f"henn_search_{p}", [f"-DHENN_PART={p}"]) for p in range(4)],
           ("henn_build.hip", "henn_build", []), ("henn_knn.hip", "henn_knn", []),
           ("henn_serve.hip", "henn_serve", [])]
ARCH = os.environ.get("HENN_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
         "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
         "-I", os.path.join(os.path.dirname(HERE), "include")]


def _compile(job) -> str:
    src, name, extra = job
    obj = os.path.join(BUILD, name + ".o")
    cmd = ["hipcc", *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} {' '.join(extra)}:\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-Wl,--no-undefined", *objs,
           "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
