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
SOURCES = ["sqa_kernels.hip", "team_kernels.hip", "pt_kernels.hip", "decode_kernels.hip", "noalloc.hip", "host_core.cpp", "api_sqa.cpp",
           "api_pt.cpp", "api_server.cpp"]
CALIB_SOURCES = ["calib_kernels.hip"]
# Per-file flags.  The team kernel (one replica per workgroup, often a single wave) and the PT
# kernel (one workgroup per ladder) run latency-bound loops that are sensitive to where the loops
# start: with 64-byte aligned loops the N = 8 ME and LHZ single-handle anneals went from 5.35 and
# 5.96 ms to 5.26 and 5.89 ms and the 256-ladder PT launch from 0.3294 to 0.3268 s.  The same flag
# on sqa_kernels.hip made the batched sweep kernel 0.2-0.4 % slower, so it is not used there.
_ALIGN = ["-falign-loops=64"]
FILE_FLAGS = {"team_kernels.hip": _ALIGN, "pt_kernels.hip": _ALIGN, "decode_kernels.hip": _ALIGN}
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
        cmd = [hipcc()] + common + FILE_FLAGS.get(src, []) + lang + ["-c", path, "-o", obj]
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


HOST_SOURCES = ["host_core.cpp", "api_sqa.cpp", "api_pt.cpp", "api_server.cpp"]


def build_host_sanitized(out_dir: str, verbose: bool = False) -> str:
    """libsqa_asan.so in out_dir: the library's host code (embedding, layout, tables,
    handle and server bookkeeping) built with AddressSanitizer and
    UndefinedBehaviorSanitizer, linked with the device objects of the last build()
    (the kernels are not instrumented).  Load it through SQA_LIBRARY with clang's
    ASan runtime preloaded."""
    build_dir = os.path.join(HERE, "_build")
    dev_objs = [os.path.join(build_dir, s + ".o") for s in SOURCES if s.endswith(".hip")]
    missing = [o for o in dev_objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"run build() first: missing {missing}")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "-fvisibility=hidden", f"--offload-arch={ARCH}", "-ffp-contract=off"]
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(out_dir, src + ".asan.o")
        cmd = [hipcc()] + common + san + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    lib = os.path.join(out_dir, "libsqa_asan.so")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-shared-libsan"] + san + ["-o", lib] + objs + \
        dev_objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
