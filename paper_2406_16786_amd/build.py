"""Build the HIP library ``libsphbuf.so`` for gfx950 in-tree.

hipcc compiles the kernels and the C ABI (``csrc/sphbuf.hip``) and the host FP64
geometry (``csrc/geometry.cpp``); both are linked into one shared library next to
this file.  FP contraction is off everywhere so the FP64 recheck evaluates each
product and sum separately.

Packed FP32 instructions are switched off for the device code with the target
feature ``-packed-fp32-ops``.  hipcc hands the flag to the host pass as well,
which does not know the feature and says so ("not a recognized feature for this
target"); the device pass honours it.  That is checked on every build: the
device assembly of ``sphbuf.hip`` is generated with the same flags and the build
fails if it holds any ``v_pk_*_f32`` instruction.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsphbuf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-I", os.path.join(ROOT, "include"),
          "-I", CSRC]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
PACKED_FP32 = re.compile(r"^\s*v_pk_\w*_f32\b", re.MULTILINE)


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def check_no_packed_fp32(asm_path: str) -> int:
    """Number of packed FP32 instructions in a device assembly file (must be 0)."""
    with open(asm_path) as f:
        return len(PACKED_FP32.findall(f.read()))


def build(verbose: bool = False, extra_flags=None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    extra = list(extra_flags or [])
    geo_o = os.path.join(BUILD, "geometry.o")
    hip_o = os.path.join(BUILD, "sphbuf.o")
    hip_s = os.path.join(BUILD, "sphbuf-" + ARCH + ".s")
    _run([HIPCC, *COMMON, "-x", "c++", "-c", os.path.join(CSRC, "geometry.cpp"), "-o", geo_o], verbose)
    _run([HIPCC, *COMMON, *DEVICE, *extra, "-c", os.path.join(CSRC, "sphbuf.hip"), "-o", hip_o], verbose)
    _run([HIPCC, *COMMON, *DEVICE, *extra, "--cuda-device-only", "-S", os.path.join(CSRC, "sphbuf.hip"), "-o",
          hip_s], verbose)
    n_pk = check_no_packed_fp32(hip_s)
    if n_pk:
        raise RuntimeError(f"{hip_s}: {n_pk} packed FP32 instructions in the device code")
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, hip_o, geo_o], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
