"""Compile libblink.so for gfx950 in-tree (hipcc), after regenerating the twiddle tables."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libblink.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep packed-FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


PROBES = os.path.join(PKG, "probes")


def build_probes(verbose: bool = False) -> None:
    """The measurement probes under csrc/probes (stand-alone executables)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(PROBES, exist_ok=True)
    flags = [f for f in HIPCC_FLAGS if f not in ("-fPIC", "-shared")]
    for src in sorted(os.listdir(os.path.join(CSRC, "probes"))):
        if not src.endswith(".hip"):
            continue
        exe = os.path.join(PROBES, src[:-4])
        cmd = [hipcc, *flags, "-I", CSRC, os.path.join(CSRC, "probes", src), "-o", exe]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    sys.path.insert(0, CSRC)
    try:
        import gen_twiddles
        gen_twiddles.main()
    finally:
        sys.path.pop(0)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "blink_api.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    build_probes(verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
