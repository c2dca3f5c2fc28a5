"""The optional diffusive flux on the GPU vs the oracle (GPU).

With PPM_DIFFUSION every face where the flow converges gains the diffusive
flux of the sweep input (Sec. "Hydrodynamics: The PPM method", after CW84),
on the Riemann flux and on the HLL fallback flux, in every sweep kernel, in
the capture of coarse fluxes for flux correction, and in both solvers.  FP64
must agree with the oracle bit for bit (fields, timesteps, registers, event
counts); mixed precision by relative L1.  Captured graphs of the HLLC and
diffusion builds replay exactly what the same steps give when launched
eagerly.
"""
import numpy as np
import pytest

from oracle import amr
from paper_1307_2265_amd import workloads as W
from tests.helpers import (FIELDS, from_device, oracle_grid, stored_inputs, to_device,
                           to_device_flat)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    from paper_1307_2265_amd import ppm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ppm.lib()
    return ppm


@pytest.mark.parametrize("tiles", [None, "lanes=1", "lanes=0", "lanes=7",
                                   "block=64 lanes_block=64 tail_round=320"])
@pytest.mark.parametrize("hllc", [False, True])
def test_single_patch_equals_oracle(P, O, tiles, hllc):
    import torch
    pr = P.PPM_FP64
    d = stored_inputs(W.random_grid(40, 28, 20, 3150, W.SHOCKED), pr)
    flags = P.PPM_ALL_FLAGS | P.PPM_DIFFUSION | (P.PPM_HLLC if hllc else 0)
    print(f"tiles {tiles} hllc {hllc}", flush=True)
    patch = to_device(d, pr, with_reg=True)
    plan = P.Plan([patch], 1, pr, P.params(flags=flags), tile_config=tiles)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    G = oracle_grid(O, d, with_reg=True)
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
    assert plan.ppm_event_counts() == tuple(cnt)
    for f in FIELDS:
        assert np.array_equal(g[f], getattr(G, f)), f
    assert np.array_equal(patch.flux_reg.cpu().numpy(), G.flux_reg)
    plan.close()


@pytest.mark.parametrize("tiles", [None, "persistent=0", "persistent=0 lanes=0",
                                   "persistent=0 lanes=0 group=0"])
def test_batch_equals_oracle(P, O, tiles):
    import torch
    pr = P.PPM_FP64
    specs = W.patch_specs(40, 3160)
    nlev = 7
    fields = [stored_inputs(W.patch_fields(sp), pr) for sp in specs]
    patches = to_device_flat(fields, pr, [(sp.dx,) * 3 for sp in specs],
                             [sp.level for sp in specs], with_reg=True)
    flags = P.PPM_ALL_FLAGS | P.PPM_DIFFUSION
    plan = P.Plan(patches, nlev, pr, P.params(flags=flags), tile_config=tiles)
    dt = torch.zeros(nlev, dtype=torch.float64, device="cuda")
    grids = [oracle_grid(O, f, dx=(sp.dx,) * 3, with_reg=True) for f, sp in zip(fields, specs)]
    prm = O.params(flags=flags)
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


def test_w_cycle_with_diffusion_equals_oracle(P, O):
    # the coarse fluxes captured for flux correction carry the diffusive flux
    from tests.test_gpu_amr_step import NESTED
    pr = P.PPM_FP64
    flags = P.PPM_ALL_FLAGS | P.PPM_DIFFUSION
    fields, dxs = [], []
    for i, (lev, _, _, dims) in enumerate(NESTED):
        fields.append(stored_inputs(W.random_grid(*dims, 3170 + i, W.SHOCKED, ghost=4), pr))
        dxs.append((1.0 / 16 * 0.5 ** lev,) * 3)
    patches = [to_device(f, pr, ghost=4, dx=dx, level=lev, with_reg=lev > 0)
               for f, dx, (lev, *_) in zip(fields, dxs, NESTED)]
    h = P.Amr(patches, [(par, 2, start) for _, par, start, _ in NESTED], 3, pr,
              P.params(flags=flags))
    H = amr.Hierarchy([amr.Node(oracle_grid(O, f, ghost=4, dx=dx, with_reg=lev > 0), lev, par,
                                start, 2)
                       for f, dx, (lev, par, start, _) in zip(fields, dxs, NESTED)],
                      [O.params(flags=flags)] * 3)
    for step in range(2):
        n0 = len(H.dts)
        H.evolve()
        h.ppm_amr_step()
        assert h.ppm_amr_step_log() == H.dts[n0:], step
    for i, (p, node) in enumerate(zip(patches, H.nodes)):
        g = from_device(p)
        for f in FIELDS:
            assert np.array_equal(g[f], getattr(node.grid, f)), (i, f)
    h.close()


def test_mixed_precision_l1(P, O):
    import torch
    pr = P.PPM_MIXED
    d = stored_inputs(W.random_grid(32, 32, 32, 3180, W.SHOCKED), pr)
    flags = P.PPM_ALL_FLAGS | P.PPM_DIFFUSION
    patch = to_device(d, pr)
    plan = P.Plan([patch], 1, pr, P.params(flags=flags))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.ppm_fill_periodic()
    plan.ppm_cfl_dt(dt)
    plan.ppm_step(dt, 0)
    torch.cuda.synchronize()
    g = from_device(patch)
    plan.close()
    G = oracle_grid(O, d)
    O.fill_periodic(G)
    O.step(G, O.params(flags=flags), float(dt.item()), 0)
    act = (slice(3, -3),) * 3
    for f in FIELDS:
        ref = getattr(G, f)[act]
        l1 = np.abs(g[f][act] - ref).sum() / np.abs(ref).sum()
        print(f"mixed with diffusion {f}: relative L1 {l1:.2e}")
        assert l1 <= 1e-5, f


@pytest.mark.parametrize("extra", ["diffusion", "hllc", "hllc+diffusion"])
def test_graph_replays_equal_eager_steps(P, extra):
    # one captured graph per sweep order (fill + step with the next dt),
    # replayed with eager work between the replays, against the same steps
    # launched eagerly: fields and timesteps identical after every step
    import torch
    flags = P.PPM_ALL_FLAGS
    if "diffusion" in extra:
        flags |= P.PPM_DIFFUSION
    if "hllc" in extra:
        flags |= P.PPM_HLLC
    print(f"graph {extra}", flush=True)
    d = W.random_grid(40, 24, 16, 3210, W.SHOCKED)
    A, B = to_device(d, P.PPM_FP64), to_device(d, P.PPM_FP64)
    pa = P.Plan([A], 1, P.PPM_FP64, P.params(flags=flags))
    pb = P.Plan([B], 1, P.PPM_FP64, P.params(flags=flags))
    dta = torch.zeros(1, dtype=torch.float64, device="cuda")
    dtb = torch.zeros(1, dtype=torch.float64, device="cuda")
    graphs = [P.Graph(pb, dtb, order, P.PPM_GRAPH_FILL | P.PPM_GRAPH_STEP_CFL)
              for order in (0, 1)]
    pa.ppm_fill_periodic()
    pa.ppm_cfl_dt(dta)
    pb.ppm_fill_periodic()
    pb.ppm_cfl_dt(dtb)
    for s in range(4):
        pa.ppm_fill_periodic()
        pa.ppm_step_cfl(dta, s % 2)
        graphs[s % 2].ppm_graph_launch()
        torch.cuda.synchronize()
        junk = torch.ones(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(dta, dtb), s
        for f in FIELDS:
            assert torch.equal(getattr(A, f), getattr(B, f)), (s, f)
    del junk
    for g in graphs:
        g.close()
    pa.close()
    pb.close()
