"""Builds the gfx950 library paper_1603_03755_amd/libsqa.so with hipcc, and
beside it libsqa_calib.so, the benchmark's VALU issue-rate probe (not part of
the library's interface).

Usage: python -m paper_1603_03755_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsqa.so")
CALIB_LIB = os.path.join(HERE, "libsqa_calib.so")
SOURCES = ["sqa_kernels.hip", "pt_kernels.hip", "decode_kernels.hip", "noalloc.hip", "host_core.cpp", "api_sqa.cpp",
           "api_pt.cpp", "api_server.cpp"]
CALIB_SOURCES = ["calib_kernels.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _link(sources, lib, build_dir, common, verbose):
    objs = []
    for src in sources:
        path = os.path.join(CSRC, src)
        obj = os.path.join(build_dir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc()] + common + lang + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", "-Wall", "-Wno-unused-result", f"--offload-arch={ARCH}",
              "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    _link(SOURCES, LIB, build_dir, common, verbose)
    _link(CALIB_SOURCES, CALIB_LIB, build_dir, common, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
