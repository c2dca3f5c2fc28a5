"""Build libppm.so (HIP, gfx950) in-tree with hipcc.

The whole library is compiled with -ffp-contract=off and without fast-math:
double-precision results are then fixed by IEEE-754 and the order the source
writes each expression in.  Packed FP32 instructions are disabled
(-packed-fp32-ops).

ppm_kernels.hip is compiled four times (PPM_KERNEL_PASS 1 to 4), so that
each group of sweep kernels takes the LLVM machine scheduler that runs it
fastest on gfx950 (measured, alternating runs on one box): iterative-ilp for
the double-precision marching sweeps (and every non-sweep kernel) and for
the mixed-precision lane-parallel ones, max-ilp for the mixed-precision
marching sweeps and for the double-precision lane-parallel ones (under
iterative-ilp their last-sweep build spills four times as much in its
loop).  Against the default scheduler: 512^3 grid about -1 % (FP64) and
-2.4 % (mixed) per step, 4096-patch batch -1 % and -2 %.  Scheduling
reorders instructions only, so results are unchanged bit for bit.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libppm.so")
# (source, object, extra flags)
UNITS = [
    ("ppm_kernels.hip", "ppm_kernels_fp64.o",
     ["-DPPM_KERNEL_PASS=1", "-mllvm", "--amdgpu-sched-strategy=iterative-ilp"]),
    ("ppm_kernels.hip", "ppm_kernels_mixed.o",
     ["-DPPM_KERNEL_PASS=2", "-mllvm", "--amdgpu-sched-strategy=max-ilp"]),
    ("ppm_kernels.hip", "ppm_kernels_fp64_lanes.o",
     ["-DPPM_KERNEL_PASS=3", "-mllvm", "--amdgpu-sched-strategy=max-ilp"]),
    ("ppm_kernels.hip", "ppm_kernels_mixed_lanes.o",
     ["-DPPM_KERNEL_PASS=4", "-mllvm", "--amdgpu-sched-strategy=iterative-ilp"]),
    ("ppm_api.cpp", "ppm_api.o", []),
    ("ppm_amr.cpp", "ppm_amr.o", []),
    ("ppm_noalloc.cpp", "ppm_noalloc.o", []),
]
SOURCES = sorted({u[0] for u in UNITS})
ARCH = os.environ.get("PPM_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wno-unused-function", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, save_temps: str | None = None) -> str:
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src, oname, extra in UNITS:
        obj = os.path.join(build_dir, oname)
        cmd = [HIPCC, "-c", *COMMON, "-x", "hip", *DEVICE, *extra]
        if src.endswith(".hip") and save_temps:
            cmd += [f"-save-temps={save_temps}", "-Rpass-analysis=kernel-resource-usage"]
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
