"""Build the HIP library ``libmlfma.so`` in-tree for gfx950.

Host-only C++ (tree construction, FP64 precompute) is compiled with g++;
the kernels and the C ABI with hipcc.  Objects go to ``_build/`` at the
repository root.  Run as ``python -m paper_2006_15367_amd.build``.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmlfma.so")

HOST_SOURCES = ["tree.cpp", "operators.cpp"]
HIP_SOURCES = ["kernels.hip", "m2l.hip", "interp.hip", "fused.hip", "pair.hip", "solver.hip",
               "fft.hip", "capi.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are kept out of every kernel.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", "-I", INCLUDE, "-I", CSRC]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-pthread", "-I", INCLUDE, "-I",
              CSRC, "-I", "/opt/rocm/include"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(jobs=4):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    procs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmd = ["g++"] + HOST_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmd = [HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = False
    for cmd, p in procs:
        if p.wait() != 0:
            print("FAILED:", " ".join(cmd), file=sys.stderr, flush=True)
            failed = True
    if failed:
        raise RuntimeError("HIP library build failed")
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
         + ["-pthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
