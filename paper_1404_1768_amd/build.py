"""Build the gfx950 shared library ``libfeast_mi355x.so`` in-tree with hipcc.

Usage: ``python -m paper_1404_1768_amd.build`` (or ``build()`` from Python).
Objects go to ``_build/`` at the repository root; the library is written next
to this file, where the binding loads it.
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
OBJDIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libfeast_mi355x.so")
ARCH = "gfx950"

DEVICE_SOURCES = ["k_gemm.hip", "k_lu.hip", "k_misc.hip", "k_band.hip"]
HOST_HIP_SOURCES = ["feast.cpp", "batch.cpp"]           # host code that calls the HIP runtime
HOST_SOURCES = ["host_eig.cpp", "host_util.cpp", "host_sparse.cpp"]   # plain C++

COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC, "-fcx-limited-range"]
# Packed-FP32 instructions are disabled for every device compile.
DEVICE_FLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops", "-munsafe-fp-atomics"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "unknown target feature" not in l and "packed-fp32-ops" not in l
                    and l.strip() != "1 warning generated." and l.strip())
    if r.returncode != 0:
        raise RuntimeError("command failed: %s\n%s" % (" ".join(cmd), r.stdout))
    return out


def build(verbose: bool = False, jobs: int = 8) -> str:
    hipcc = _hipcc()
    os.makedirs(OBJDIR, exist_ok=True)
    jobs_list = []
    for src in DEVICE_SOURCES:
        obj = os.path.join(OBJDIR, src + ".o")
        jobs_list.append([hipcc, *COMMON, *DEVICE_FLAGS, "-x", "hip", "-c",
                          os.path.join(CSRC, src), "-o", obj])
    for src in HOST_HIP_SOURCES:
        obj = os.path.join(OBJDIR, src + ".o")
        jobs_list.append([hipcc, *COMMON, *DEVICE_FLAGS, "-x", "hip", "-c",
                          os.path.join(CSRC, src), "-o", obj])
    for src in HOST_SOURCES:
        obj = os.path.join(OBJDIR, src + ".o")
        jobs_list.append(["g++", "-O3", "-std=c++17", "-fPIC", "-march=x86-64-v3",
                          "-fcx-limited-range", "-I" + CSRC, "-c", os.path.join(CSRC, src),
                          "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        outs = list(ex.map(_run, jobs_list))
    if verbose:
        for o in outs:
            if o:
                print(o)
    objs = [c[-1] for c in jobs_list]
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
