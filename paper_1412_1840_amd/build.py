"""Builds libqmi.so (the HIP library behind include/qmi.h) in-tree for gfx950.

    python -m paper_1412_1840_amd.build [--verbose]

hipcc compiles the device code for gfx950 only, with packed-FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops; the host pass warns that it does not know the
feature, which is harmless).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqmi.so")
SOURCES = ["qmi_kernels.hip", "qmi_search.hip", "qmi_bands.hip", "qmi_prep.hip", "qmi_api.hip"]
PROBE = os.path.join(HERE, "valu_rates")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    # -ffp-contract=off: no implicit fused multiply-add, so that frequency grid points
    # f0 + k * df are rounded twice exactly as the definition states (explicit fma() calls in the
    # kernels are unaffected).
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + flags() + ["-shared", "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    # The VALU rate probe (an executable of its own; bench.py runs it to measure the roofline).
    ptmp = PROBE + ".tmp%d" % os.getpid()
    res = subprocess.run([hipcc()] + flags() + ["-o", ptmp, os.path.join(CSRC, "valu_rates.hip")],
                         stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed (valu_rates):\n" + res.stdout)
    os.replace(ptmp, PROBE)
    return LIB


if __name__ == "__main__":
    build(verbose="--verbose" in sys.argv)
    print(LIB)
