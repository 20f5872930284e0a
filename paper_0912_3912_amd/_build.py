"""Build the HIP library ``libsg.so`` in-tree for gfx950 with hipcc.

Every source is compiled to its own object in parallel (``_build/``), then the
objects are linked into the shared library."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsg.so")
OBJDIR = os.path.join(PKG, "_build")

SOURCES = ["sg_host.cpp", "sg_bnb.cpp", "sg_kernels.hip", "sg_lattice.hip", "sg_batch.hip", "sg_queue.hip",
           "sg_msc.hip", "sg_fm.hip", "sg_fm_lanes.hip", "sg_fm_big.hip", "sg_dense.hip", "sg_bits.hip", "sg_wide.hip", "sg_noalloc.hip"]
HEADERS = ["sg_layout.h", "sg_launch.h", "sg_device.h"]

# Packed-FP32 instructions are disabled for all device code (the path is
# integer-only anyway).
HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16, len(SOURCES)))


def build(verbose: bool = False) -> str:
    """Compile every source and link libsg.so (always recompiles)."""
    os.makedirs(OBJDIR, exist_ok=True)
    tag = "%d" % os.getpid()
    objs = [os.path.join(OBJDIR, src.replace(".", "_") + "." + tag + ".o") for src in SOURCES]

    def compile_one(src: str, obj: str) -> None:
        cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    tmp = LIB + ".tmp" + tag
    try:
        with ThreadPoolExecutor(max_workers=_jobs()) as ex:
            list(ex.map(compile_one, SOURCES, objs))
        cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    finally:
        # this build's objects go whether it succeeded or not
        for o in objs:
            try:
                os.remove(o)
            except OSError:
                pass
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
