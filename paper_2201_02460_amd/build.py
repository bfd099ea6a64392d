"""Build ``libepi.so`` (gfx950 HIP kernels + C++ host runtime) in-tree with hipcc.

    python -m paper_2201_02460_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD, "libepi.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# (source, object, extra flags): kernels.hip is compiled a second time with
# EPI_SCAN_CHECK for the checking instantiations of the scan kernel
SOURCES = [("kernels.hip", "kernels.o", []), ("kernels.hip", "kernels_check.o", ["-DEPI_SCAN_CHECK"]),
           ("runtime.cpp", "runtime.o", []), ("server.cpp", "server.o", [])]
# Packed FP32 VALU instructions are disabled for all device code.
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5", "-Xclang",
         "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument", f"-I{INCLUDE}", "-Wall"]


def _compile(entry):
    src, obj, extra = entry
    out = os.path.join(BUILD, obj)
    lang = [] if src.endswith(".hip") else ["-x", "hip"]
    cmd = [HIPCC, *FLAGS, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", out]
    subprocess.run(cmd, check=True)
    return out


def build(verbose=False):
    """Compile every source and link ``_build/libepi.so``; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp, "-lpthread"], check=True)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
