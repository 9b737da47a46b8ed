"""Build step of the gfx950 library: hipcc -> paper_2303_13435_amd/libultima.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libultima.so")
SOURCES = ["ur_kernels.hip", "ur_mixed.hip", "ur_noalloc.hip", "ur_api.cpp"]
# ur_kernels.hip is compiled once per part (-DUR_PART=k): each part
# instantiates one group of transform passes, so the parts build in parallel
KERNEL_PARTS = 11
HEADERS = ["ur_device.hpp", "ur_geom.hpp", "ur_kernels.hpp", "ur_tuned.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("UR_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are kept out of every kernel (some of their forms
# have produced wrong results on this hardware); -O3 would otherwise emit them.
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def _compile_one(src: str, obj: str, defines=()) -> None:
    cmd = [HIPCC] + FLAGS + list(defines) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")


def build(verbose: bool = True) -> str:
    """Compile every HIP source for gfx950 and link the shared library."""
    import concurrent.futures as cf
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    for src in SOURCES:
        stem = os.path.splitext(src)[0]
        if src == "ur_kernels.hip":
            for k in range(KERNEL_PARTS):
                jobs.append((src, os.path.join(objdir, f"{stem}.p{k}.o"), (f"-DUR_PART={k}",)))
        else:
            jobs.append((src, os.path.join(objdir, stem + ".o"), ()))
    objs = [j[1] for j in jobs]
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "0")) or (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(lambda j: _compile_one(*j), jobs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + objs + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libultima.so failed")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
