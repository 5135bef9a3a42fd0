"""Build the HIP library (libacq.so) for gfx950, in-tree.

Each HIP source is compiled by hipcc for --offload-arch=gfx950 with packed FP32
instructions disabled; the host-only C++ source by g++; everything is linked
into paper_2005_10445_amd/libacq.so.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libacq.so")

HIP_SOURCES = ["kernels.hip", "correlate.hip", "plan.hip", "learned_kernels.hip", "cnn.hip", "fsk.hip"]
CXX_SOURCES = ["host_logic.cpp"]
ARCH = os.environ.get("ACQ_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC, "-Wall"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False, out: str = LIB, build_dir: str = BUILD, csrc: str = CSRC) -> str:
    os.makedirs(build_dir, exist_ok=True)
    jobs = []
    objs = []
    hip_flags = [f if f != CSRC else csrc for f in HIP_FLAGS]
    cxx_flags = [f if f != CSRC else csrc for f in CXX_FLAGS]
    for src in HIP_SOURCES:
        obj = os.path.join(build_dir, src + ".o")
        objs.append(obj)
        jobs.append([HIPCC, *hip_flags, "-c", os.path.join(csrc, src), "-o", obj])
    for src in CXX_SOURCES:
        obj = os.path.join(build_dir, src + ".o")
        objs.append(obj)
        jobs.append(["g++", *cxx_flags, "-c", os.path.join(csrc, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr, file=sys.stderr)
    tmp = out + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
