"""AMR level step (W-cycle) on the GPU vs the oracle (GPU).

ppm_amr_step runs EvolveLevel over a static hierarchy: per-level CFL
timesteps with subcycling, ghost zones from the parent blended in time and
from siblings, the coarse fluxes through child footprints recorded during the
coarse sweeps, the fine registers summed over substeps, flux correction and
projection (Secs. "Adaptive Mesh Refinement", "Flux correction",
"Projection").  FP64 must reproduce the oracle's W-cycle (oracle/amr.py) bit
for bit: the sequence of (level, dt) steps, every field of every patch,
ghosts included, every flux register and the event counts, over two root
steps; the composite totals of the nested hierarchy are conserved to
round-off.  Mixed precision is checked by per-field relative L1.
"""
import numpy as np
import pytest

from oracle import amr
from paper_1307_2265_amd import workloads as W
from tests.helpers import FIELDS, from_device, oracle_grid, stored_inputs, to_device

pytestmark = pytest.mark.gpu

# (level, parent, start, dims): nested with a non-touching sibling (ghost 4),
# and three levels with abutting siblings (ghost 3)
NESTED = [(0, -1, (0, 0, 0), (16, 16, 16)),
          (1, 0, (8, 8, 8), (12, 12, 12)),
          (2, 1, (20, 20, 20), (8, 8, 8)),
          (1, 0, (2, 22, 4), (8, 6, 10))]
ABUTTING = [(0, -1, (0, 0, 0), (16, 16, 16)),
            (1, 0, (6, 6, 6), (10, 8, 8)),
            (1, 0, (16, 6, 6), (8, 8, 8)),
            (1, 0, (6, 14, 6), (12, 6, 8)),
            (2, 1, (16, 16, 16), (8, 8, 8)),
            (2, 1, (24, 16, 16), (6, 6, 6))]


@pytest.fixture(scope="module")
def P():
    import torch
    from paper_1307_2265_amd import ppm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ppm.lib()
    return ppm


def _setup(P, O, spec, ghost, seed, recipe, prec, flags=None):
    fields, dxs = [], []
    for i, (lev, _, _, dims) in enumerate(spec):
        fields.append(stored_inputs(W.random_grid(*dims, seed + i, recipe, ghost=ghost), prec))
        dxs.append((1.0 / 16 * 0.5 ** lev,) * 3)
    patches = [to_device(f, prec, ghost=ghost, dx=dx, level=lev, with_reg=lev > 0)
               for f, dx, (lev, *_) in zip(fields, dxs, spec)]
    prm = P.params() if flags is None else P.params(flags=flags)
    h = P.Amr(patches, [(par, 2, start) for _, par, start, _ in spec], 1 + max(s[0] for s in spec),
              prec, prm)
    oprm = O.params() if flags is None else O.params(flags=flags)
    nodes = [amr.Node(oracle_grid(O, f, ghost=ghost, dx=dx, with_reg=lev > 0), lev, par, start, 2)
             for f, dx, (lev, par, start, _) in zip(fields, dxs, spec)]
    H = amr.Hierarchy(nodes, [oprm] * (1 + max(s[0] for s in spec)))
    return patches, h, H


@pytest.mark.parametrize("case", ["nested", "nested-hllc", "nested-shocked", "abutting"])
def test_w_cycle_equals_oracle_fp64(P, O, case):
    # nested-shocked: level 1 steps four times per root step, its child once per
    # level-1 step, and the child's sweeps meet near-vacuum edge states
    spec, ghost, recipe, seed = {"abutting": (ABUTTING, 3, W.SHOCKED, 600),
                                 "nested-shocked": (NESTED, 4, W.SHOCKED, 3170)}.get(
                                     case, (NESTED, 4, W.GENTLE, 600))
    flags = P.PPM_ALL_FLAGS | P.PPM_HLLC if case == "nested-hllc" else None
    print(f"case {case}", flush=True)
    patches, h, H = _setup(P, O, spec, ghost, seed, recipe, P.PPM_FP64, flags)
    for step in range(2):
        n0 = len(H.dts)
        H.evolve()
        h.ppm_amr_step()
        assert h.ppm_amr_step_log() == H.dts[n0:], step
    t, n = h.ppm_amr_times()
    assert t == H.t and n == H.nsteps
    for i, (p, node) in enumerate(zip(patches, H.nodes)):
        g = from_device(p)
        for f in FIELDS:
            assert np.array_equal(g[f], getattr(node.grid, f)), (i, f)
        if p.flux_reg is not None:
            assert np.array_equal(p.flux_reg.cpu().numpy(), node.grid.flux_reg), i
    print(f"{case}: steps per level {n}, events {h.ppm_amr_event_counts()}")
    h.close()


def test_w_cycle_conserves_composite_totals_on_the_gpu(P, O):
    patches, h, H = _setup(P, O, NESTED, 4, 610, W.GENTLE, P.PPM_FP64)
    # the composite totals of the device state, in the oracle's bookkeeping
    def totals():
        for p, node in zip(patches, H.nodes):
            g = from_device(p)
            for f in FIELDS:
                getattr(node.grid, f)[...] = g[f]
        return H.composite_totals()
    t0 = totals()
    h.ppm_amr_step()
    h.ppm_amr_step()
    t1 = totals()
    scale = np.array([t0[0], t0[0], t0[0], t0[0], t0[4]])
    assert np.all(np.abs(t1 - t0) <= 1e-13 * scale), (t1 - t0) / scale
    h.close()


def test_w_cycle_mixed_precision_l1(P, O):
    patches, h, H = _setup(P, O, NESTED, 4, 620, W.GENTLE, P.PPM_MIXED)
    H.evolve()
    h.ppm_amr_step()
    assert [lv for lv, _ in h.ppm_amr_step_log()] == [lv for lv, _ in H.dts]
    for i, (p, node) in enumerate(zip(patches, H.nodes)):
        g = from_device(p)
        gh = p.ghost
        act = (slice(gh, -gh),) * 3
        for f in FIELDS:
            ref = getattr(node.grid, f)[act]
            l1 = np.abs(g[f][act] - ref).sum() / np.abs(ref).sum()
            assert l1 <= 1e-5, (i, f, l1)
    h.close()


def test_shock_pool_w_cycle_equals_oracle(P, O):
    # the paper's shock pool (inflow and outflow root faces, static refined
    # region): 25 root steps, bit for bit
    import torch
    from tests.test_oracle_amr import _shock_pool
    H, _ = _shock_pool(O, True)
    patches = []
    for lev, node in enumerate(H.nodes):
        g = node.grid
        d = {f: getattr(g, f).copy() for f in FIELDS}
        patches.append(to_device(d, P.PPM_FP64, ghost=g.ghost, dx=(g.dx, g.dy, g.dz), level=lev,
                                 with_reg=lev > 0))
    h = P.Amr(patches, [(-1, 2, (0, 0, 0)), (0, 2, (50, 2, 2))], 2, P.PPM_FP64,
              P.params(gamma=1.4), root_kinds=H.root_kinds, root_inflow=H.root_inflow)
    for step in range(25):
        n0 = len(H.dts)
        H.evolve()
        h.ppm_amr_step()
        assert h.ppm_amr_step_log() == H.dts[n0:], step
    torch.cuda.synchronize()
    for i, (p, node) in enumerate(zip(patches, H.nodes)):
        g = from_device(p)
        for f in FIELDS:
            assert np.array_equal(g[f], getattr(node.grid, f)), (i, f)
    h.close()


def test_wave_pool_w_cycle_equals_oracle(P, O):
    # the paper's wave pool (a short linear sound wave through a static refined
    # region, outflow root faces): 40 root steps, bit for bit
    import torch
    from tests.test_oracle_amr import _wave_pool
    H, _ = _wave_pool(O, True)
    patches = []
    for lev, node in enumerate(H.nodes):
        g = node.grid
        d = {f: getattr(g, f).copy() for f in FIELDS}
        patches.append(to_device(d, P.PPM_FP64, ghost=g.ghost, dx=(g.dx, g.dy, g.dz), level=lev,
                                 with_reg=lev > 0))
    h = P.Amr(patches, [(-1, 2, (0, 0, 0)), (0, 2, (50, 2, 2))], 2, P.PPM_FP64,
              P.params(gamma=1.4), root_kinds=H.root_kinds)
    for step in range(40):
        n0 = len(H.dts)
        H.evolve()
        h.ppm_amr_step()
        assert h.ppm_amr_step_log() == H.dts[n0:], step
    torch.cuda.synchronize()
    for i, (p, node) in enumerate(zip(patches, H.nodes)):
        g = from_device(p)
        for f in FIELDS:
            assert np.array_equal(g[f], getattr(node.grid, f)), (i, f)
        assert i == 0 or np.array_equal(p.flux_reg.cpu().numpy(), node.grid.flux_reg), i
    h.close()


def test_w_cycle_with_gravity_and_expansion_equals_oracle(P, O):
    # every patch with an acceleration field, each level its own a and adot
    import torch
    patches, h, H = _setup(P, O, NESTED, 4, 630, W.GENTLE, P.PPM_FP64)
    h.close()
    expand = [(1.3, 0.4), (1.31, 0.41), (1.32, 0.42)]
    for i, (p, node) in enumerate(zip(patches, H.nodes)):
        acc = W.acceleration_field(p.rho.shape, 640 + i, 2.0)
        node.grid.accel = acc
        p.accel = tuple(torch.from_numpy(a).to("cuda") for a in acc)
    H.params = [O.params(a=a, adot=ad) for a, ad in expand]
    H.expansion = True
    h = P.Amr(patches, [(par, 2, start) for _, par, start, _ in NESTED], 3, P.PPM_FP64,
              P.params())
    h.ppm_amr_set_expansion(torch.tensor([v for av in expand for v in av], dtype=torch.float64,
                                         device="cuda"))
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


def test_w_cycle_bench_hierarchy_one_root_step(P, O):
    # The benchmark's W-cycle workload (128^3 periodic root, 64 level-1 blocks
    # of 32^3, 512 level-2 blocks of 24^3, gentle fields) in its launch
    # configuration: one root step (1 + 2 + 5 level steps) against the
    # oracle's, bit for bit on every patch.
    print("generating the nested hierarchy", flush=True)
    hier = W.nested_hierarchy(128, (32, 24), (4, 2))
    fields = [stored_inputs(W.random_grid(*h.dims, 5000 + i, W.GENTLE), P.PPM_FP64)
              for i, h in enumerate(hier)]
    dxs = [(0.5 ** h.level / 128,) * 3 for h in hier]
    patches = [to_device(f, P.PPM_FP64, dx=dx, level=h.level, with_reg=h.level > 0)
               for f, dx, h in zip(fields, dxs, hier)]
    h = P.Amr(patches, [(x.parent, 2, x.start) for x in hier], 3, P.PPM_FP64)
    H = amr.Hierarchy([amr.Node(oracle_grid(O, f, dx=dx, with_reg=x.level > 0), x.level,
                                x.parent, x.start, 2)
                       for f, dx, x in zip(fields, dxs, hier)], [O.params()] * 3)
    print("oracle root step", flush=True)
    H.evolve()
    print("gpu root step", flush=True)
    h.ppm_amr_step()
    assert h.ppm_amr_step_log() == H.dts
    bad = [i for i, (p, node) in enumerate(zip(patches, H.nodes))
           if any(not np.array_equal(from_device(p)[f], getattr(node.grid, f)) for f in FIELDS)]
    print(f"patches: {len(patches)}, not bitwise equal: {len(bad)}")
    assert not bad
    h.close()
