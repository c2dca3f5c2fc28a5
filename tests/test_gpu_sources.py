"""Gravity source terms and comoving coordinates on the GPU vs the oracle (GPU).

A patch with an acceleration field gets the time-centred gravitational
sources of Eqs. momentum_diff and energy_diff in every sweep; with expansion
factors set (ppm_set_expansion), every sweep divides its flux differences and
its gravity source by the level's a, the CFL timestep is kappa a / max
signal, and ppm_expansion integrates the split expansion terms (Sec.
"Physical Equations").  FP64 must agree with the oracle bit for bit (fields,
timesteps and event counts), on one patch through every sweep kernel and on
batches of uneven patches with per-level expansion factors; mixed precision
is checked by relative L1 after a step, and the expansion step alone, which
only scales stored values, bit for bit after narrowing.
"""
import numpy as np
import pytest

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


def _dev(arrs, dtype):
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=dtype).contiguous()
                 for a in arrs)


def _stored_accel(shape, seed, prec, P, amp=3.0):
    acc = W.acceleration_field(shape, seed, amp)
    if prec == P.PPM_MIXED:
        acc = tuple(a.astype(np.float32).astype(np.float64) for a in acc)
    return acc


@pytest.mark.parametrize("tiles", [None, "lanes=1", "lanes=0", "lanes=7",
                                   "block=64 lanes_block=64 tail_round=320"])
@pytest.mark.parametrize("hllc", [False, True])
def test_single_patch_gravity_and_expansion_equal_oracle(P, O, tiles, hllc):
    import torch
    pr = P.PPM_FP64
    d = stored_inputs(W.random_grid(40, 28, 20, 3100, W.SHOCKED), pr)
    acc = _stored_accel(d["rho"].shape, 3101, pr, P)
    a, adot = 1.7, 0.6
    flags = P.PPM_ALL_FLAGS | (P.PPM_HLLC if hllc else 0)
    print(f"tiles {tiles} hllc {hllc}", flush=True)
    patch = to_device(d, pr)
    patch.accel = _dev(acc, torch.float64)
    plan = P.Plan([patch], 1, pr, P.params(flags=flags), tile_config=tiles)
    expand = torch.tensor([a, adot], dtype=torch.float64, device="cuda")
    plan.ppm_set_expansion(expand)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    G = oracle_grid(O, d)
    G.accel = acc
    prm = O.params(flags=flags, a=a, adot=adot)
    cnt = [0, 0]
    for s in range(4):
        plan.ppm_fill_periodic()
        plan.ppm_cfl_dt(dt)
        plan.ppm_step(dt, s % 2)
        plan.ppm_expansion(dt)
        O.fill_periodic(G)
        dto = O.cfl_dt(G, prm)
        c = O.step(G, prm, dto, s % 2)
        O.expansion(G, prm, dto)
        cnt[0] += c.fallback_faces
        cnt[1] += c.floored_cells
        torch.cuda.synchronize()
        assert float(dt.item()) == dto, s
    g = from_device(patch)
    assert plan.ppm_event_counts() == tuple(cnt)
    plan.close()
    for f in FIELDS:
        assert np.array_equal(g[f], getattr(G, f)), f


def test_gravity_without_expansion_and_static_plan_unchanged(P, O):
    # gravity alone (a = 1, no ppm_set_expansion), and a plan without a field
    # next to it: the latter must give the oracle's static step
    import torch
    pr = P.PPM_FP64
    d = stored_inputs(W.random_grid(24, 20, 16, 3200, W.SHOCKED), pr)
    acc = _stored_accel(d["rho"].shape, 3201, pr, P)
    pg, ps = to_device(d, pr), to_device(d, pr)
    pg.accel = _dev(acc, torch.float64)
    plg, pls = P.Plan([pg], 1, pr, P.params()), P.Plan([ps], 1, pr, P.params())
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    Gg, Gs = oracle_grid(O, d), oracle_grid(O, d)
    Gg.accel = acc
    prm = O.params()
    for s in range(3):
        for plan, G in ((plg, Gg), (pls, Gs)):
            plan.ppm_fill_periodic()
            plan.ppm_cfl_dt(dt)
            plan.ppm_step(dt, s % 2)
            O.fill_periodic(G)
            dto = O.cfl_dt(G, prm)
            O.step(G, prm, dto, s % 2)
            torch.cuda.synchronize()
            assert float(dt.item()) == dto
    for p, G in ((pg, Gg), (ps, Gs)):
        g = from_device(p)
        for f in FIELDS:
            assert np.array_equal(g[f], getattr(G, f)), f
    plg.close()
    pls.close()


def _batch_with_sources(P, prec, specs, seed, tiles):
    """A batch of uneven patches (views into shared arrays, accelerations
    likewise) with per-level expansion factors."""
    import torch
    fields = [stored_inputs(W.patch_fields(sp), prec) for sp in specs]
    accs = [_stored_accel(f["rho"].shape, seed + i, prec, P) for i, f in enumerate(fields)]
    patches = to_device_flat(fields, prec, [(sp.dx,) * 3 for sp in specs],
                             [sp.level for sp in specs], with_reg=True)
    low = torch.float32 if prec == P.PPM_MIXED else torch.float64
    flat = [torch.from_numpy(np.concatenate([a[k].ravel() for a in accs])).to("cuda", dtype=low)
            for k in range(3)]
    off = 0
    for p, f in zip(patches, fields):
        n = f["rho"].size
        p.accel = tuple(t[off:off + n].view(f["rho"].shape) for t in flat)
        off += n
    return fields, accs, patches


EXPAND7 = [(1.0 + 0.15 * l, 0.3 + 0.05 * l) for l in range(7)]


@pytest.mark.parametrize("tiles", [None, "persistent=0", "persistent=0 lanes=0",
                                   "persistent=0 lanes=0 group=0"])
def test_batch_with_per_level_expansion_equals_oracle(P, O, tiles):
    import torch
    pr = P.PPM_FP64
    specs = W.patch_specs(40, 3300)
    nlev = 7
    fields, accs, patches = _batch_with_sources(P, pr, specs, 3400, tiles)
    print(f"tiles {tiles}", flush=True)
    plan = P.Plan(patches, nlev, pr, P.params(), tile_config=tiles)
    expand = torch.tensor([v for av in EXPAND7 for v in av], dtype=torch.float64, device="cuda")
    plan.ppm_set_expansion(expand)
    dt = torch.zeros(nlev, dtype=torch.float64, device="cuda")
    grids = [oracle_grid(O, f, dx=(sp.dx,) * 3, with_reg=True) for f, sp in zip(fields, specs)]
    for G, acc in zip(grids, accs):
        G.accel = acc
    prms = [O.params(a=a, adot=ad) for a, ad in EXPAND7]
    cnt = [0, 0]
    for s in range(2):
        plan.ppm_cfl_dt(dt)
        plan.ppm_step(dt, s % 2)
        plan.ppm_expansion(dt)
        torch.cuda.synchronize()
        smax = np.zeros(nlev)
        for G, sp in zip(grids, specs):
            smax[sp.level] = max(smax[sp.level], O.cfl_signal_max(G, prms[sp.level]))
        dto = np.array([(prms[l].cfl * prms[l].a) / smax[l] if smax[l] > 0 else np.inf
                        for l in range(nlev)])
        assert np.array_equal(dt.cpu().numpy(), dto), (s, dt, dto)
        for G, sp in zip(grids, specs):
            c = O.step(G, prms[sp.level], float(dto[sp.level]), s % 2)
            O.expansion(G, prms[sp.level], float(dto[sp.level]))
            cnt[0] += c.fallback_faces
            cnt[1] += c.floored_cells
    assert plan.ppm_event_counts() == tuple(cnt)
    act = (slice(3, -3),) * 3
    for i, (p, G) in enumerate(zip(patches, grids)):
        g = from_device(p)
        for f in FIELDS:
            assert np.array_equal(g[f][act], getattr(G, f)[act]), (i, f)
        assert np.array_equal(p.flux_reg.cpu().numpy(), G.flux_reg), i
    plan.close()


@pytest.mark.parametrize("tiles", [None, "persistent=0 lanes=0"])
def test_step_with_next_dt_equals_step_then_cfl_under_expansion(P, tiles):
    # the fused next-dt of ppm_step_cfl takes the level's a like ppm_cfl_dt
    import torch
    pr = P.PPM_FP64
    specs = W.patch_specs(40, 3500)
    nlev = 7
    expand = torch.tensor([v for av in EXPAND7 for v in av], dtype=torch.float64, device="cuda")
    _, _, A = _batch_with_sources(P, pr, specs, 3600, tiles)
    _, _, B = _batch_with_sources(P, pr, specs, 3600, tiles)
    pa = P.Plan(A, nlev, pr, P.params(), tile_config=tiles)
    pb = P.Plan(B, nlev, pr, P.params(), tile_config=tiles)
    pa.ppm_set_expansion(expand)
    pb.ppm_set_expansion(expand)
    dta = torch.zeros(nlev, dtype=torch.float64, device="cuda")
    dtb = torch.zeros(nlev, dtype=torch.float64, device="cuda")
    pb.ppm_cfl_dt(dtb)
    for s in range(3):
        pa.ppm_cfl_dt(dta)
        assert torch.equal(dta, dtb), s
        pa.ppm_step(dta, s % 2)
        pb.ppm_step_cfl(dtb, s % 2)
        torch.cuda.synchronize()
        for x, y in zip(A, B):
            for f in FIELDS:
                assert torch.equal(getattr(x, f), getattr(y, f)), (s, f)
    pa.close()
    pb.close()


def test_graph_replays_equal_eager_steps_with_sources(P):
    import torch
    pr = P.PPM_FP64
    d = stored_inputs(W.random_grid(32, 24, 16, 3700, W.SHOCKED), pr)
    acc = _stored_accel(d["rho"].shape, 3701, pr, P)
    expand = torch.tensor([1.4, 0.5], dtype=torch.float64, device="cuda")
    pe, pg = to_device(d, pr), to_device(d, pr)
    pe.accel = _dev(acc, torch.float64)
    pg.accel = _dev(acc, torch.float64)
    plan_e, plan_g = P.Plan([pe], 1, pr, P.params()), P.Plan([pg], 1, pr, P.params())
    plan_e.ppm_set_expansion(expand)
    plan_g.ppm_set_expansion(expand)
    dte = torch.zeros(1, dtype=torch.float64, device="cuda")
    dtg = torch.zeros(1, dtype=torch.float64, device="cuda")
    graph = P.Graph(plan_g, dtg, 0, P.PPM_GRAPH_FILL | P.PPM_GRAPH_CFL | P.PPM_GRAPH_STEP)
    for s in range(3):
        plan_e.ppm_fill_periodic()
        plan_e.ppm_cfl_dt(dte)
        plan_e.ppm_step(dte, 0)
        plan_e.ppm_expansion(dte)
        graph.ppm_graph_launch()
        plan_g.ppm_expansion(dtg)
        torch.cuda.synchronize()
        assert torch.equal(dte, dtg), s
        for f in FIELDS:
            assert torch.equal(getattr(pe, f), getattr(pg, f)), (s, f)
    graph.close()
    plan_e.close()
    plan_g.close()


def test_mixed_precision_step_with_sources_l1(P, O):
    import torch
    pr = P.PPM_MIXED
    d = stored_inputs(W.random_grid(32, 32, 32, 3800, W.GENTLE), pr)
    acc = _stored_accel(d["rho"].shape, 3801, pr, P)
    a, adot = 1.3, 0.4
    patch = to_device(d, pr)
    patch.accel = _dev(acc, torch.float32)
    plan = P.Plan([patch], 1, pr, P.params())
    plan.ppm_set_expansion(torch.tensor([a, adot], dtype=torch.float64, device="cuda"))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.ppm_fill_periodic()
    plan.ppm_cfl_dt(dt)
    plan.ppm_step(dt, 0)
    plan.ppm_expansion(dt)
    torch.cuda.synchronize()
    g = from_device(patch)
    plan.close()
    G = oracle_grid(O, d)
    G.accel = acc
    prm = O.params(a=a, adot=adot)
    O.fill_periodic(G)
    dto = O.cfl_dt(G, prm)
    assert float(dt.item()) == pytest.approx(dto, rel=1e-5)
    O.step(G, prm, float(dt.item()), 0)
    O.expansion(G, prm, float(dt.item()))
    act = (slice(3, -3),) * 3
    for f in FIELDS:
        ref = getattr(G, f)[act]
        l1 = np.abs(g[f][act] - ref).sum() / np.abs(ref).sum()
        print(f"mixed with sources {f}: relative L1 {l1:.2e}")
        assert l1 <= 1e-5, f


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_expansion_step_alone_equals_oracle(P, O, prec):
    import torch
    pr = P.PPM_FP64 if prec == "fp64" else P.PPM_MIXED
    specs = W.patch_specs(12, 3900)
    nlev = 7
    fields = [stored_inputs(W.patch_fields(sp), pr) for sp in specs]
    patches = to_device_flat(fields, pr, [(sp.dx,) * 3 for sp in specs],
                             [sp.level for sp in specs])
    plan = P.Plan(patches, nlev, pr, P.params(gamma=1.4))
    with pytest.raises(RuntimeError, match="no expansion"):
        plan.ppm_expansion(torch.zeros(nlev, dtype=torch.float64, device="cuda"))
    plan.ppm_set_expansion(torch.tensor([v for av in EXPAND7 for v in av], dtype=torch.float64,
                                        device="cuda"))
    dts = np.array([0.01 * (l + 1) for l in range(nlev)])
    plan.ppm_expansion(torch.tensor(dts, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    for i, (p, f, sp) in enumerate(zip(patches, fields, specs)):
        g = from_device(p)
        G = oracle_grid(O, f, dx=(sp.dx,) * 3)
        a, ad = EXPAND7[sp.level]
        O.expansion(G, O.params(gamma=1.4, a=a, adot=ad), float(dts[sp.level]))
        for k in FIELDS:
            ref = getattr(G, k)
            if pr == P.PPM_MIXED and k not in ("etot", "eint"):
                ref = ref.astype(np.float32).astype(np.float64)
            assert np.array_equal(g[k], ref), (i, k)
    plan.close()


def test_full_size_512_step_with_sources_in_bench_configuration(P, O):
    # The benchmark's gravity + comoving workload: the shocked 512^3 grid with
    # a seeded acceleration field and a = 1.7, adot = 0.6, in its launch
    # configuration (autotuned tiles, the gravity builds); one step (CFL, the
    # three sweeps, the expansion terms) against the oracle cell by cell.
    import torch
    from paper_1307_2265_amd import autotune
    n = 512
    cfg = W.WORKLOADS["shocked512"]
    print("generating 512^3 input", flush=True)
    d = stored_inputs(W.random_grid(n, n, n, cfg["seed"], cfg["recipe"]), P.PPM_FP64)
    acc = W.acceleration_field(d["rho"].shape, 4242, 3.0)
    a, adot = 1.7, 0.6
    print("oracle step", flush=True)
    G = oracle_grid(O, d)
    G.accel = acc
    prm = O.params(a=a, adot=adot)
    O.fill_periodic(G)
    dto = O.cfl_dt(G, prm)
    c = O.step(G, prm, dto, 0)
    O.expansion(G, prm, dto)
    print("gpu step", flush=True)
    patch = to_device(d, P.PPM_FP64)
    patch.accel = _dev(acc, torch.float64)
    del acc
    plan = P.Plan([patch], 1, P.PPM_FP64, P.params(),
                  tile_config=autotune.best_tiles("single/fp64"))
    plan.ppm_set_expansion(torch.tensor([a, adot], dtype=torch.float64, device="cuda"))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.ppm_fill_periodic()
    plan.ppm_cfl_dt(dt)
    plan.ppm_step(dt, 0)
    plan.ppm_expansion(dt)
    torch.cuda.synchronize()
    assert float(dt.item()) == dto
    assert plan.ppm_event_counts() == (c.fallback_faces, c.floored_cells)
    for f in FIELDS:
        g = getattr(patch, f)[3:-3, 3:-3, 3:-3].cpu().numpy()
        differ = int(np.count_nonzero(g != getattr(G, f)[3:-3, 3:-3, 3:-3]))
        print(f"{f}: cells not bitwise equal {differ}")
        assert differ == 0, f
    plan.close()
