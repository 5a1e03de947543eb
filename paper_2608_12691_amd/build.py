"""Build libalchnb.so (HIP, gfx950) in-tree.

    python -m paper_2608_12691_amd.build [--force]

Each translation unit is compiled with hipcc for gfx950 only; packed FP32
instructions are disabled (-packed-fp32-ops).  The shared library lands next
to this file as ``libalchnb.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libalchnb.so")
BUILD_DIR = os.path.join(ROOT, "_build", "alchnb")
SOURCES = ["alch_nb.cpp", "list_kernels.hip", "tile_kernels.hip", "aux_kernels.hip", "ldyn_kernels.hip",
           "hrex_kernels.hip", "noalloc.hip", "pme_kernels.hip"]
HEADERS = ["anb_internal.h", "anb_kernels.h", "dihedral_cv.h", "erfc_coeffs.h", "lane_ops.h", "pair_math.h"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
            "-packed-fp32-ops", "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def _compile(src: str) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), "-c", os.path.join(CSRC, src), "-o", obj] + common_flags()
    if src.endswith(".cpp"):
        cmd = [hipcc(), "-c", os.path.join(CSRC, src), "-o", obj, "-O2", "-std=c++17", "-fPIC", "-I", INCLUDE,
               "-I", CSRC, "-Wall"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every translation unit and link libalchnb.so (always rebuilds when force)."""
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    if not force and os.path.exists(OUT):
        newest = max(os.path.getmtime(os.path.join(CSRC, f)) for f in srcs + HEADERS
                     if os.path.exists(os.path.join(CSRC, f)))
        newest = max(newest, os.path.getmtime(os.path.join(INCLUDE, "alch_nb.h")))
        if os.path.getmtime(OUT) >= newest:
            return OUT
    with cf.ThreadPoolExecutor(max_workers=min(4, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-o", tmp] + objs + ["--offload-arch=" + ARCH, "-fPIC"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(force="--no-force" not in sys.argv, verbose=True)
