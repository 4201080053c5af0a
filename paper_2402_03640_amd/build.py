"""Build the HIP library ``libhipmsat.so`` in-tree for gfx950.

Host plan code is compiled with g++, the kernels and the C ABI with hipcc
(cross-compiles without a GPU).  ``python -m paper_2402_03640_amd.build``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "libhipmsat.so")
BUILD = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", INC, "-I", CSRC]
# Packed FP32 instructions are kept out of the device code; contraction into
# FMA is off so every schedule rounds identically.
HIP_FLAGS = COMMON + [f"--offload-arch={ARCH}", "-ffp-contract=off",
                      "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                      "-Wno-unused-command-line-argument"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = [
        ["g++"] + COMMON + ["-ffp-contract=off", "-c", os.path.join(CSRC, "plan.cpp"), "-o",
                            os.path.join(BUILD, "plan.o")],
        [HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, "kernels.hip"), "-o",
                               os.path.join(BUILD, "kernels.o")],
        [HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, "hipmsat.hip"), "-o",
                               os.path.join(BUILD, "hipmsat.o")],
        [HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, "small.hip"), "-o",
                               os.path.join(BUILD, "small.o")],
    ]
    with ThreadPoolExecutor(4) as ex:
        outs = list(ex.map(_run, jobs))
    tmp = OUT + ".tmp"
    outs.append(_run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
                      os.path.join(BUILD, "plan.o"), os.path.join(BUILD, "kernels.o"),
                      os.path.join(BUILD, "hipmsat.o"), os.path.join(BUILD, "small.o")]))
    os.replace(tmp, OUT)
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
