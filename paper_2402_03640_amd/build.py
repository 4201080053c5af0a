"""Build the HIP library ``libhipmsat.so`` (and the bandwidth probes,
``libhipmsat_probe.so``) in-tree for gfx950.

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
PROBE_OUT = os.path.join(PKG, "libhipmsat_probe.so")
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


SAN_DIR = os.path.join(BUILD, "san")
# gcc's AddressSanitizer and UndefinedBehaviorSanitizer for the host-only plan
# builder (the HIP sources stay as they are: one sanitizer runtime per process)
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


def _gcc_runtime_dir() -> str:
    return os.path.dirname(subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip())


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Build libhipmsat.so in the package; with ``sanitize`` a copy whose
    host plan code carries ASan/UBSan, in _build/san/ (load it through the
    HIPMSAT_LIB variable, with gcc's libasan and libubsan preloaded)."""
    os.makedirs(BUILD, exist_ok=True)
    bdir = SAN_DIR if sanitize else BUILD
    os.makedirs(bdir, exist_ok=True)
    out = os.path.join(SAN_DIR, "libhipmsat.so") if sanitize else OUT
    plan_flags = SAN_FLAGS if sanitize else []
    jobs = [
        ["g++"] + COMMON + plan_flags + ["-ffp-contract=off", "-c", os.path.join(CSRC, "plan.cpp"), "-o",
                                         os.path.join(bdir, "plan.o")],
        [HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, "kernels.hip"), "-o",
                               os.path.join(BUILD, "kernels.o")],
        [HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, "hipmsat.hip"), "-o",
                               os.path.join(BUILD, "hipmsat.o")],
        [HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, "small.hip"), "-o",
                               os.path.join(BUILD, "small.o")],
    ]
    if not sanitize:
        jobs.append([HIPCC] + HIP_FLAGS + ["-shared", os.path.join(CSRC, "probe.hip"), "-o", PROBE_OUT + ".tmp"])
    with ThreadPoolExecutor(4) as ex:
        outs = list(ex.map(_run, jobs))
    tmp = out + ".tmp"
    san_link = []
    if sanitize:
        rt = _gcc_runtime_dir()
        san_link = ["-L" + rt, "-Wl,-rpath," + rt, "-lasan", "-lubsan"]
    outs.append(_run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
                      os.path.join(bdir, "plan.o"), os.path.join(BUILD, "kernels.o"),
                      os.path.join(BUILD, "hipmsat.o"), os.path.join(BUILD, "small.o")] + san_link))
    os.replace(tmp, out)
    if not sanitize:
        os.replace(PROBE_OUT + ".tmp", PROBE_OUT)
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
