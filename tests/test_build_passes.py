"""The kernel source compiled in several passes (build.py): every kernel is
emitted by exactly one pass, and the passes together emit each sweep kernel
family of both precisions (CPU only; reads the objects of the last build)."""
import os
import re
import shutil
import subprocess

import pytest

from paper_1307_2265_amd import build

KERNEL = re.compile(r"\bppm::(?:__device_stub__)?([a-z_]+_kernel)\b")


def _kernel_stubs(obj):
    out = subprocess.run(["nm", "-C", "--defined-only", obj], check=True, capture_output=True,
                         text=True).stdout
    stubs = set()
    for line in out.splitlines():
        parts = line.split(None, 2)
        if len(parts) == 3 and parts[1] in "tTwW" and KERNEL.search(parts[2]):
            stubs.add(parts[2])
    return stubs


def test_each_kernel_emitted_by_exactly_one_pass():
    if shutil.which("nm") is None:
        pytest.skip("nm not available")
    bdir = os.path.join(build.HERE, "_build")
    objs = [os.path.join(bdir, o) for src, o, _ in build.UNITS if src == "ppm_kernels.hip"]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("no kernel objects: run build() first")
    assert len(objs) == 4
    seen = {}
    for o in objs:
        for stub in _kernel_stubs(o):
            assert stub not in seen, (stub, seen.get(stub), o)
            seen[stub] = o
    families = {KERNEL.search(s).group(1) + ("/mixed" if "PrecMixed" in s else "/fp64" if "PrecF64" in s else "")
                for s in seen}
    for fam in ("sweep_kernel", "sweep_split_kernel", "sweep_lanes_kernel", "sweep_tail_kernel",
                "batch_persistent_kernel", "capture_kernel", "fill_from_parent_kernel"):
        assert fam + "/fp64" in families and fam + "/mixed" in families, fam
    assert "cfl_finalize_kernel" in families and "accumulate_kernel" in families
