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


@pytest.mark.parametrize("tiles", [None, "lanes=1", "lanes=0", "lanes=7",
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


def _mixed_floor(x):
    """The floor a PPM_MIXED plan uses: the nearest float at or above x."""
    f = np.float32(x)
    if float(f) < x:
        f = np.nextafter(f, np.float32(np.inf))
    return float(f)


def test_mixed_precision_stays_physical_and_tracks_the_oracle(P, O):
    """Near-vacuum cells are beyond what float reconstruction resolves: the
    interface value between a cell of density 1 and one at the floor (1e-20)
    carries an absolute rounding error near 1e-8, so the vacuum side of such a
    stencil, and the states traced from it, are wrong by many orders of
    magnitude relative to their own size, more faces need the HLL fallback
    and more cells the floors than in double.  What holds is that the mixed
    path stays finite and above the floors, and that the mass, momentum and
    energy it carries track the oracle's; the L1 it reaches on this input is
    stated below as a regression bound (a few times the measured values),
    not the bound of the benchmark workloads (no cells at the floors there),
    which the other mixed-precision tests hold to 1e-5 per step."""
    import torch
    pr = P.PPM_MIXED
    prm = P.params()
    floor = _mixed_floor(prm.rho_floor)
    d = W.vacuum_pockets(W.random_grid(14, 12, 10, 3192, W.SHOCKED, ghost=GH), 3193,
                         rho_vac=floor, p_vac=floor, ghost=GH)
    d = stored_inputs(d, pr)
    patch = to_device(d, pr, ghost=GH)
    plan = P.Plan([patch], 1, pr, prm)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    G = oracle_grid(O, d, ghost=GH)
    po = O.params()
    act = (slice(GH, -GH),) * 3
    l1 = []
    for s in range(4):
        # both take the oracle's timestep, so the comparison sees only precision
        O.fill_periodic(G)
        dto = O.cfl_dt(G, po)
        O.step(G, po, dto, s % 2)
        plan.ppm_fill_periodic()
        dt.fill_(dto)
        plan.ppm_step(dt, s % 2)
        torch.cuda.synchronize()
        g = from_device(patch)
        o = {f: getattr(G, f)[act] for f in FIELDS}
        m = {f: g[f][act] for f in FIELDS}
        # density, and the conserved rho v, rho E, rho e
        err = {"rho": float(np.abs(m["rho"] - o["rho"]).sum() / np.abs(o["rho"]).sum())}
        for f in FIELDS[1:]:
            cm, co = m["rho"] * m[f], o["rho"] * o[f]
            err[f] = float(np.abs(cm - co).sum() / np.abs(co).sum())
        l1.append(err)
    plan.close()
    print("mixed near-vacuum L1 of rho, rho v, rho E, rho e per step:", l1, flush=True)
    for f in FIELDS:
        assert np.isfinite(g[f][act]).all(), f
    assert g["rho"][act].min() >= floor
    assert g["eint"][act].min() > 0.0
    bound = {"rho": 2e-4, "vx": 1e-2, "vy": 1e-2, "vz": 1e-2, "etot": 1e-2, "eint": 5e-2}
    for s in range(4):
        for f in FIELDS:
            assert l1[s][f] <= bound[f], (s, f, l1[s][f])
