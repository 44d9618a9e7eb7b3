"""Build the GP-MOOD HIP library (libgpmood.so) in-tree for gfx950.

Every call compiles from source:
  * gp_weights.cpp with g++ (host, __float128 + libquadmath),
  * the .hip sources with hipcc --offload-arch=gfx950, FP contraction off (the
    kernels write every fma explicitly) and packed FP32 instructions disabled,
  * linked into paper_2110_08683_amd/libgpmood.so.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libgpmood.so")

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
             "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
HIP_SOURCES = ["gpmood_kernels.hip", "gpmood_abi.hip", "gpmood_batch.hip", "gpmood_adjoint.hip", "gpmood3d.hip"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout)
        raise RuntimeError(f"build step failed: {cmd[0]} {cmd[-1]}")
    return r.stdout


def build(verbose=False, extra_hip_flags=()):
    os.makedirs(BUILD, exist_ok=True)
    jobs = [["g++", "-O2", "-std=c++17", "-fPIC", "-fno-fast-math", "-I", CSRC, "-c",
             os.path.join(CSRC, "gp_weights.cpp"), "-o", os.path.join(BUILD, "gp_weights.o")]]
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        jobs.append([HIPCC, *HIP_FLAGS, *extra_hip_flags, "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o:
                sys.stdout.write(o)
    objs = [os.path.join(BUILD, "gp_weights.o")] + [os.path.join(BUILD, s.replace(".hip", ".o")) for s in HIP_SOURCES]
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lquadmath"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
