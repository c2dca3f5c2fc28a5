"""Near-vacuum cells on the GPU vs the oracle (GPU).

Cells at the density and pressure floors moving fast through dense shocked
gas drive the reconstructed edge density or pressure to zero, so the
characteristic tracing (Sec. "Hydrodynamics: The PPM method", CW84 Eqs.
3.5-3.7) meets a zero sound speed: the oracle's IEEE arithmetic then carries
a zero, an infinity or a NaN through the correction terms, and the floors and
the HLL fallback take over.  FP64 must still agree with the oracle bit for
bit (fields, timesteps, event counts) in every sweep kernel, with the
two-shock and the HLLC solver, single patch and batched; mixed precision must
stay finite and above the floors.
"""
import numpy as np
import pytest

from paper_1307_2265_amd import workloads as W
from tests.helpers import (FIELDS, from_device, oracle_grid, stored_inputs, to_device,
                           to_device_flat)

pytestmark = pytest.mark.gpu
GH = 4


@pytest.fixture(scope="module")
def P():
    import torch
    from paper_1307_2265_amd import ppm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ppm.lib()
    return ppm


def _field(seed, ghost=GH):
    return W.vacuum_pockets(W.random_grid(14, 12, 10, seed, W.SHOCKED, ghost=ghost), seed + 1,
                            ghost=ghost)


@pytest.mark.parametrize("tiles", [None, "lanes=0", "lanes=7",
                                   "block=64 lanes_block=64 tail_round=320"])
@pytest.mark.parametrize("hllc", [False, True])
def test_single_patch_equals_oracle(P, O, tiles, hllc):
    import torch
    pr = P.PPM_FP64
    d = stored_inputs(_field(3190), pr)
    flags = P.PPM_ALL_FLAGS | (P.PPM_HLLC if hllc else 0)
    print(f"tiles {tiles} hllc {hllc}", flush=True)
    patch = to_device(d, pr, ghost=GH, with_reg=True)
    plan = P.Plan([patch], 1, pr, P.params(flags=flags), tile_config=tiles)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    G = oracle_grid(O, d, ghost=GH, with_reg=True)
    prm = O.params(flags=flags)
    cnt = [0, 0]
    for s in range(4):
        plan.ppm_fill_periodic()
        plan.ppm_cfl_dt(dt)
        plan.ppm_step(dt, s % 2)
        O.fill_periodic(G)
        dto = O.cfl_dt(G, prm)
        c = O.step(G, prm, dto, s % 2)
        cnt[0] += c.fallback_faces
        cnt[1] += c.floored_cells
        torch.cuda.synchronize()
        assert float(dt.item()) == dto, s
    g = from_device(patch)
    assert cnt[0] > 0 and cnt[1] > 0  # the fallback and the floors did act
    assert plan.ppm_event_counts() == tuple(cnt)
    for f in FIELDS:
        assert np.array_equal(g[f], getattr(G, f)), f
    assert np.array_equal(patch.flux_reg.cpu().numpy(), G.flux_reg)
    plan.close()


@pytest.mark.parametrize("tiles", [None, "persistent=0"])
def test_batch_equals_oracle(P, O, tiles):
    import torch
    pr = P.PPM_FP64
    specs = W.patch_specs(24, 3200)
    nlev = 7
    fields = [stored_inputs(W.vacuum_pockets(W.patch_fields(sp), 3300 + i, ghost=3), pr)
              for i, sp in enumerate(specs)]
    patches = to_device_flat(fields, pr, [(sp.dx,) * 3 for sp in specs],
                             [sp.level for sp in specs], with_reg=True)
    plan = P.Plan(patches, nlev, pr, P.params(), tile_config=tiles)
    dt = torch.zeros(nlev, dtype=torch.float64, device="cuda")
    grids = [oracle_grid(O, f, dx=(sp.dx,) * 3, with_reg=True) for f, sp in zip(fields, specs)]
    prm = O.params()
    for s in range(2):
        plan.ppm_cfl_dt(dt)
        plan.ppm_step(dt, s % 2)
        torch.cuda.synchronize()
        dtg = dt.cpu().numpy()
        for G, sp in zip(grids, specs):
            O.step(G, prm, float(dtg[sp.level]), s % 2)
    act = (slice(3, -3),) * 3
    for i, (p, G) in enumerate(zip(patches, grids)):
        g = from_device(p)
        for f in FIELDS:
            assert np.array_equal(g[f][act], getattr(G, f)[act]), (i, f)
        assert np.array_equal(p.flux_reg.cpu().numpy(), G.flux_reg), i
    plan.close()


def test_mixed_precision_stays_physical(P):
    import torch
    pr = P.PPM_MIXED
    d = stored_inputs(_field(3192), pr)
    patch = to_device(d, pr, ghost=GH)
    prm = P.params()
    plan = P.Plan([patch], 1, pr, prm)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    for s in range(4):
        plan.ppm_fill_periodic()
        plan.ppm_cfl_dt(dt)
        plan.ppm_step(dt, s % 2)
    torch.cuda.synchronize()
    g = from_device(patch)
    plan.close()
    act = (slice(GH, -GH),) * 3
    for f in FIELDS:
        assert np.isfinite(g[f][act]).all(), f
    assert g["rho"][act].min() >= np.float32(prm.rho_floor)
    assert g["eint"][act].min() > 0.0
