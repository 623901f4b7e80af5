"""Compile libfio.so (host builder + gfx950 kernels) in-tree.

Host C++ sources are compiled with ROCm's clang++, HIP sources with hipcc for
gfx950 only; packed-FP32 instruction selection is disabled for device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfio.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")

CXX_SOURCES = ["la.cpp", "stages.cpp", "butterfly.cpp", "hif1d.cpp", "hif2d.cpp", "build.cpp"]
HIP_SOURCES = ["kernels.hip", "construct.hip", "capi.hip"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
HOST_FLAGS = ["-fcomplex-arithmetic=improved"]
HIP_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + p.stdout)
    return p.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = []
    for s in CXX_SOURCES:
        jobs.append([CLANGXX, *COMMON, *HOST_FLAGS, "-c", os.path.join(CSRC, s),
                     "-o", os.path.join(OBJ, s + ".o")])
    for s in HIP_SOURCES:
        jobs.append([HIPCC, *COMMON, *HIP_FLAGS, "-c", os.path.join(CSRC, s),
                     "-o", os.path.join(OBJ, s + ".o")])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [os.path.join(OBJ, s + ".o") for s in CXX_SOURCES + HIP_SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp, "-lpthread",
          "-L" + os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx", "-lrocsolver", "-lrocblas", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    os.replace(tmp, LIB)
    # the C ABI from plain C: a file-to-file solve (HIP runtime C API for device memory)
    ex = os.path.join(HERE, "fio_solve_file")
    _run(["gcc", "-O2", "-std=c99", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROOT, "include"),
          "-I" + os.path.join(ROCM, "include"), os.path.join(HERE, "examples", "solve_file.c"),
          "-L" + HERE, "-lfio", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
          "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lm", "-o", ex + ".tmp"])
    os.replace(ex + ".tmp", ex)
    # measurement aid (copy kernel of known size, MFMA rates)
    cal = os.path.join(HERE, "fio_calibrate")
    _run([HIPCC, "-O3", "-std=c++17", *HIP_FLAGS, os.path.join(CSRC, "calibrate.hip"),
          "-o", cal + ".tmp"])
    os.replace(cal + ".tmp", cal)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
