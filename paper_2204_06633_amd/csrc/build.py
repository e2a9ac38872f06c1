"""Build the HIP library ``_lisaresp.so`` for gfx950 in the package directory.

Run ``python -m paper_2204_06633_amd.csrc.build`` (or call ``build()``).  Every
call recompiles.  Flags: -O3, C++17, no fast-math (IEEE division and square
root), FMA contraction allowed, packed-FP32 instructions disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
TARGET = os.path.join(PKG, "_lisaresp.so")
SOURCES = (["forward_%s.hip" % k for k in "abcd"] + ["adjoint_%s.hip" % k for k in "abcd"] +
           ["batchfwd%d_%s.hip" % (g, k) for g in (1, 2) for k in "abcd"] +
           ["batchadj_%s.hip" % k for k in "abcd"] +
           ["util.hip", "fd_kernels.hip", "gb_kernels.hip", "dispatch.cpp", "api.cpp", "api_batch.cpp",
            "api_fd.cpp", "api_gb.cpp", "api_noalloc.hip"])
ARCH = os.environ.get("LR_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    return ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-munsafe-fp-atomics", "-fno-fast-math", "-Wall", "-Wno-unused-variable",
            "-I" + os.path.join(ROOT, "include")]


def build(verbose=True, jobs=None, target=TARGET, defines=(), out_dir=None):
    """Compile every source to an object in parallel, then link the library.
    ``defines``: extra -D options (tuning macros such as LR_PROJ_MIN_WAVES),
    for variant libraries built to ``target`` with objects in ``out_dir``."""
    out_dir = out_dir or os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    cc = hipcc()
    t0 = time.time()
    jobs = jobs or min(os.cpu_count() or 4, int(os.environ.get("MAX_JOBS", "8")), 16)
    objs = [os.path.join(out_dir, src.rsplit(".", 1)[0] + ".o") for src in SOURCES]
    pending = list(zip(SOURCES, objs))
    running = []
    while pending or running:
        while pending and len(running) < jobs:
            src, obj = pending.pop(0)
            cmd = [cc, *flags(), *["-D" + d for d in defines], "-c", os.path.join(HERE, src),
                   "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((src, subprocess.Popen(cmd)))
        src, p = running.pop(0)
        if p.wait() != 0:
            for _, q in running:
                q.wait()
            raise RuntimeError("compilation of %s failed" % src)
    tmp = target + ".tmp%d" % os.getpid()
    cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, target)
    if verbose:
        print("built %s in %.1f s" % (target, time.time() - t0), flush=True)
    return target


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
