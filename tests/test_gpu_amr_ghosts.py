"""AMR patch ghost fill on the GPU vs the oracle (GPU).

ppm_set_hierarchy + ppm_fill_ghosts: SecondOrderA interpolation of the
parent's conserved quantities into every ghost cell of a patch, then the copy
from siblings whose active region covers a ghost cell (Sec. "Boundary
conditions", Appendix "Interpolation").  A three-level hierarchy with abutting
and ghost-overlapping siblings is filled level by level on both sides; FP64
must agree bit for bit everywhere, and in mixed precision the GPU interpolates
in FP64 from the same stored values, so its FP32 density and velocities are
the oracle's values narrowed to FP32.
"""
import numpy as np
import pytest

from paper_1307_2265_amd import workloads as W
from tests.helpers import FIELDS, from_device, oracle_grid, stored_inputs, to_device

pytestmark = pytest.mark.gpu

G = 3
# (level, parent, start, dims): level-1 cells are half the root's, level-2 half of level 1
HIER = [
    (0, -1, (0, 0, 0), (16, 16, 16)),
    (1, 0, (6, 6, 6), (10, 8, 8)),      # A
    (1, 0, (16, 6, 6), (8, 8, 8)),      # B: abuts A along +x
    (1, 0, (6, 14, 6), (12, 6, 8)),     # C: abuts A along +y, inside B's ghosts at a corner
    (2, 1, (16, 16, 16), (8, 8, 8)),    # D inside A
    (2, 1, (24, 16, 16), (6, 6, 6)),    # E abuts D along +x, inside A
]


@pytest.fixture(scope="module")
def P():
    import torch
    from paper_1307_2265_amd import ppm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ppm.lib()
    return ppm


def _fields(pr, seed):
    out = []
    for i, (lev, _, _, dims) in enumerate(HIER):
        d = W.random_grid(*dims, seed + i, W.SHOCKED)
        out.append(stored_inputs(d, pr))
    return out


def _oracle(O, fields, stored32=False):
    """The oracle's fill, level by level; stored32: the device keeps density and
    velocities in FP32, so a filled level is narrowed before the next one
    interpolates from it."""
    grids = [oracle_grid(O, f, dx=(0.5 ** lev,) * 3) for f, (lev, *_) in zip(fields, HIER)]
    O.fill_periodic(grids[0])
    for level in (1, 2):
        members = [i for i, h in enumerate(HIER) if h[0] == level]
        for i in members:
            par = HIER[i][1]
            O.fill_from_parent(grids[i], HIER[i][2], grids[par], HIER[par][2], 2)
        for i in members:
            for j in members:
                if j != i:
                    O.copy_from_sibling(grids[i], HIER[i][2], grids[j], HIER[j][2])
        if stored32:
            for i in members:
                for f in ("rho", "vx", "vy", "vz"):
                    a = getattr(grids[i], f)
                    a[...] = a.astype(np.float32).astype(np.float64)
    return grids


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_hierarchy_ghost_fill_equals_oracle(P, O, prec):
    import torch
    pr = P.PPM_FP64 if prec == "fp64" else P.PPM_MIXED
    fields = _fields(pr, 1200)
    patches = [to_device(f, pr, dx=(0.5 ** lev,) * 3, level=lev)
               for f, (lev, *_) in zip(fields, HIER)]
    plan = P.Plan(patches, 3, pr, P.params())
    plan.ppm_set_hierarchy([(par, 2, start) for _, par, start, _ in HIER])
    plan.ppm_fill_periodic()                 # the root is a periodic box
    plan.ppm_fill_ghosts(1)
    plan.ppm_fill_ghosts(2)
    torch.cuda.synchronize()
    got = [from_device(p) for p in patches]
    plan.close()
    grids = _oracle(O, fields, stored32=pr == P.PPM_MIXED)
    for i, (g, o) in enumerate(zip(got, grids)):
        for f in FIELDS:
            ref = getattr(o, f)
            if pr == P.PPM_MIXED and f not in ("etot", "eint"):
                ref = ref.astype(np.float32).astype(np.float64)
            assert np.array_equal(g[f], ref), (i, f, np.max(np.abs(g[f] - ref)))


def test_hierarchy_is_validated(P):
    pr = P.PPM_FP64
    fields = _fields(pr, 1300)
    patches = [to_device(f, pr, dx=(0.5 ** lev,) * 3, level=lev)
               for f, (lev, *_) in zip(fields, HIER)]
    plan = P.Plan(patches, 3, pr, P.params())
    with pytest.raises(RuntimeError, match="no hierarchy"):
        plan.ppm_fill_ghosts(1)
    bad = [(par, 2, start) for _, par, start, _ in HIER]
    bad[1] = (0, 2, (-8, 6, 6))              # A's ghosts would need cells left of the root
    with pytest.raises(RuntimeError, match="outside parent"):
        plan.ppm_set_hierarchy(bad)
    bad[1] = (2, 2, (6, 6, 6))               # parent on the same level
    with pytest.raises(RuntimeError, match="one level coarser"):
        plan.ppm_set_hierarchy(bad)
    plan.close()
