"""Build libcn.so (the HIP library behind include/cn.h) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libcn.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["cn_host.cpp", "cn_kernels.hip", "cn_noalloc.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off: ordinary float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


LIB_PHASE = os.path.join(PKG, "libcn_phase.so")


def build(verbose: bool = False, phase_clocks: bool = False) -> str:
    """Compile the sources (in parallel) and link the library. phase_clocks: the profiling build (libcn_phase.so),
    whose interval kernel sums its shader clock per phase (cn_phase_clocks)."""
    lib = LIB_PHASE if phase_clocks else LIB
    tag = "_phase" if phase_clocks else ""
    extra = ["-DCN_PHASE_CLOCKS"] if phase_clocks else []
    objs, procs = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + tag + ".o")
        cmd = [HIPCC] + [f for f in FLAGS if f != "-shared"] + extra + ["-c", "-I", os.path.join(ROOT, "include"),
                                                                       "-I", CSRC, path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for cmd, p in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, phase_clocks="--phase-clocks" in sys.argv))
