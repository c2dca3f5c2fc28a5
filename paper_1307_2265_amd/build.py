"""Build libppm.so (HIP, gfx950) in-tree with hipcc.

The whole library is compiled with -ffp-contract=off and without fast-math:
double-precision results are then fixed by IEEE-754 and the order the source
writes each expression in.  Packed FP32 instructions are disabled
(-packed-fp32-ops).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libppm.so")
SOURCES = ["ppm_kernels.hip", "ppm_api.cpp", "ppm_amr.cpp", "ppm_noalloc.cpp"]
ARCH = os.environ.get("PPM_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wno-unused-function", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, save_temps: str | None = None) -> str:
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, "-c", *COMMON]
        if src.endswith(".hip"):
            cmd += ["-x", "hip", *DEVICE]
            if save_temps:
                cmd += [f"-save-temps={save_temps}", "-Rpass-analysis=kernel-resource-usage"]
        else:
            cmd += ["-x", "hip", *DEVICE]
        cmd += [os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True, cwd=build_dir)
        objs.append(obj)
    link = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, save_temps="obj" if "--temps" in sys.argv else None)
