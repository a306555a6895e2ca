"""Compiles the HIP library libfrnn.so in-tree for gfx950.

Usage: python -m paper_2202_06929_amd.build_lib [--asm]

Flags that matter for the results:
  -ffp-contract=off                 no fused multiply-add in the distance sums
  -fno-gpu-flush-denormals-to-zero  subnormal distances are kept, as on the CPU
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                    no packed FP32 instructions are generated
"""

from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libfrnn.so")
SOURCES = [os.path.join(CSRC, "frnn_kernels.hip"), os.path.join(CSRC, "frnn_api.cpp"),
           os.path.join(CSRC, "frnn_components.hip")]
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Always recompiles libfrnn.so; returns its path."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIP_FLAGS, "-shared"]
    for src in SOURCES:
        cmd += ["-x", "hip", src]
    cmd += ["-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    if verbose and res.stderr:
        print(res.stderr, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


def device_asm(out_dir: str) -> str:
    """Writes the gfx950 assembly of the kernels (for instruction checks); returns its path."""
    os.makedirs(out_dir, exist_ok=True)
    out = os.path.join(out_dir, "frnn_kernels-gfx950.s")
    cmd = [hipcc(), *HIP_FLAGS, "--cuda-device-only", "-S", "-x", "hip", SOURCES[0], "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    if "--asm" in sys.argv:
        print(device_asm(os.path.join(PKG, "_build")))
