"""HIP path vs the oracle, element by element (GPU).

FP64: within 1e-12 relative per cell (the expressions are the same IEEE
operations in the same order, so the results are expected to be identical;
the count of cells that are not bitwise equal is reported).  Mixed precision:
per-field relative L1 error after one step within 1e-5.  Everything goes
through the C ABI (paper_1307_2265_amd.ppm).
"""
import numpy as np
import pytest

from paper_1307_2265_amd import workloads as W
from tests.helpers import (FIELDS, compare_fields, from_device, oracle_grid, stored_inputs,
                           to_device, to_device_flat)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def P():
    import torch
    from paper_1307_2265_amd import ppm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ppm.lib()
    return ppm


def _dt_tensor(n=1):
    import torch
    return torch.zeros(n, dtype=torch.float64, device="cuda")


def _run_gpu_steps(P, d, nsteps, prec, flags=None, gamma=5.0 / 3.0, ghost=3, dx=None,
                   periodic=True, orders=None, with_reg=False, dt_fixed=None, tiles=None):
    import torch
    patch = to_device(d, prec, ghost=ghost, dx=dx, with_reg=with_reg)
    prm = P.params(gamma=gamma) if flags is None else P.params(gamma=gamma, flags=flags)
    plan = P.Plan([patch], 1, prec, prm, tile_config=tiles)
    dt = _dt_tensor()
    dts = []
    for s in range(nsteps):
        if periodic:
            plan.ppm_fill_periodic()
        if dt_fixed is None:
            plan.ppm_cfl_dt(dt)
        else:
            dt.fill_(dt_fixed)
        dts.append(float(dt.item()))
        plan.ppm_step(dt, orders[s] if orders else s % 2)
    torch.cuda.synchronize()
    counts = plan.ppm_event_counts()
    out = from_device(patch)
    reg = None if patch.flux_reg is None else patch.flux_reg.cpu().numpy()
    plan.close()
    return out, dts, counts, reg


def _run_oracle_steps(O, d, nsteps, flags=None, gamma=5.0 / 3.0, ghost=3, dx=None,
                      periodic=True, orders=None, with_reg=False, dt_fixed=None):
    prm = O.params(gamma=gamma) if flags is None else O.params(gamma=gamma, flags=flags)
    G = oracle_grid(O, d, ghost=ghost, dx=dx, with_reg=with_reg)
    dts, counts = [], [0, 0]
    for s in range(nsteps):
        if periodic:
            O.fill_periodic(G)
        dt = O.cfl_dt(G, prm) if dt_fixed is None else dt_fixed
        dts.append(dt)
        c = O.step(G, prm, dt, orders[s] if orders else s % 2)
        counts[0] += c.fallback_faces
        counts[1] += c.floored_cells
    return {f: getattr(G, f) for f in FIELDS}, dts, tuple(counts), G.flux_reg


@pytest.mark.parametrize("order", [0, 1, 2, 3, 4, 5])
def test_config0_one_step_fp64(P, O, order):
    # 32^3 periodic, gentle white noise, one full step (the small parity case)
    d = W.random_grid(32, 32, 32, 1000, W.GENTLE)
    g, gdt, gcnt, _ = _run_gpu_steps(P, d, 1, P.PPM_FP64, orders=[order])
    o, odt, ocnt, _ = _run_oracle_steps(O, d, 1, orders=[order])
    assert gdt == odt  # CFL reduction is bitwise
    worst, differ = compare_fields(g, o, TOL64)
    print(f"order {order}: worst rel err {worst:.3e}, cells not bitwise equal {differ}")
    assert gcnt == ocnt


@pytest.mark.parametrize("seed", range(8))
def test_random_small_grids_fp64(P, O, seed):
    rng = np.random.default_rng(500 + seed)
    nx, ny, nz = (int(v) for v in rng.integers(1, 25, size=3))
    ghost = int(rng.choice([3, 4]))
    gamma = float(rng.uniform(1.1, 5.0 / 3.0))
    recipe = W.SHOCKED if seed % 2 else W.GENTLE
    flags = int(rng.integers(0, 16))
    orders = [int(v) for v in rng.integers(0, 6, size=2)]
    print(f"seed {seed}: dims {nx}x{ny}x{nz} ghost {ghost} gamma {gamma:.3f} flags {flags} "
          f"orders {orders}", flush=True)
    d = W.random_grid(nx, ny, nz, 9000 + seed, recipe, gamma=gamma, ghost=ghost)
    g, gdt, gcnt, _ = _run_gpu_steps(P, d, 2, P.PPM_FP64, flags=flags, gamma=gamma,
                                     ghost=ghost, orders=orders)
    o, odt, ocnt, _ = _run_oracle_steps(O, d, 2, flags=flags, gamma=gamma, ghost=ghost,
                                        orders=orders)
    assert gdt == odt
    worst, differ = compare_fields(g, o, TOL64)
    print(f"  worst rel err {worst:.3e}, cells not bitwise equal {differ}, counts {gcnt}")
    assert gcnt == ocnt


def test_flux_registers_and_seeded_ghosts_fp64(P, O):
    nx, ny, nz = 13, 9, 11
    d = W.random_grid(nx, ny, nz, 4242, W.SHOCKED, seeded_ghosts=True)
    dx = (0.1, 0.125, 0.25)
    g, _, gcnt, greg = _run_gpu_steps(P, d, 1, P.PPM_FP64, dx=dx, periodic=False,
                                      with_reg=True, dt_fixed=2e-3, orders=[1])
    o, _, ocnt, oreg = _run_oracle_steps(O, d, 1, dx=dx, periodic=False, with_reg=True,
                                         dt_fixed=2e-3, orders=[1])
    compare_fields(g, o, TOL64)
    scale = np.maximum(np.abs(oreg), np.mean(np.abs(oreg)))
    assert np.max(np.abs(greg - oreg) / scale) <= TOL64
    assert gcnt == ocnt


@pytest.mark.parametrize("tiles", [None, "lanes=1", "lanes=0", "lanes=0 split=0", "lanes=7"])
def test_hll_fallback_fires_identically(P, O, tiles):
    # Vacuum-generating double rarefaction along y in a 3-D box; the
    # two-shock update first goes non-positive after about a dozen steps.
    nx, ny, nz = 4, 100, 3
    g3 = 3
    shape = (nz + 6, ny + 6, nx + 6)
    y = (np.arange(ny + 6) - g3 + 0.5) / ny
    vy = np.broadcast_to(np.where(y < 0.5, -4.0, 4.0)[None, :, None], shape).copy()
    rho = np.ones(shape)
    p = np.full(shape, 0.4)
    z = np.zeros(shape)
    st = W.stored_from_primitive(rho, z, vy, z.copy(), p, 1.4)
    d = dict(zip(FIELDS, [np.ascontiguousarray(a) for a in st]))
    dx = (0.25, 0.01, 1.0 / 3.0)
    g, _, gcnt, _ = _run_gpu_steps(P, d, 16, P.PPM_FP64, gamma=1.4, periodic=False, dx=dx,
                                   dt_fixed=0.0015, orders=[0] * 16, tiles=tiles)
    o, _, ocnt, _ = _run_oracle_steps(O, d, 16, gamma=1.4, periodic=False, dx=dx,
                                      dt_fixed=0.0015, orders=[0] * 16)
    print("fallback faces / floored cells:", gcnt, ocnt)
    assert ocnt[0] > 0
    assert gcnt == ocnt
    compare_fields(g, o, TOL64)


@pytest.mark.parametrize("recipe", ["gentle", "shocked"])
def test_mixed_precision_l1_after_one_step(P, O, recipe):
    rec = W.GENTLE if recipe == "gentle" else W.SHOCKED
    d = stored_inputs(W.random_grid(32, 32, 32, 1000, rec), P.PPM_MIXED)
    g, gdt, _, _ = _run_gpu_steps(P, d, 1, P.PPM_MIXED)
    o, odt, _, _ = _run_oracle_steps(O, d, 1)
    assert gdt == odt  # same stored inputs, CFL in double on both sides
    sl = (slice(3, -3),) * 3
    for f in FIELDS:
        l1 = np.abs(g[f][sl] - o[f][sl]).sum() / np.abs(o[f][sl]).sum()
        print(f"{recipe} {f}: relative L1 {l1:.3e}")
        assert l1 <= 1e-5, (f, l1)


def test_cfl_and_fill_match_oracle_bitwise(P, O):
    import torch
    d = W.random_grid(20, 17, 9, 77, W.SHOCKED)
    for prec in (P.PPM_FP64, P.PPM_MIXED):
        dd = stored_inputs(d, prec)
        patch = to_device(dd, prec)
        plan = P.Plan([patch], 1, prec, P.params())
        plan.ppm_fill_periodic()
        dt = _dt_tensor()
        plan.ppm_cfl_dt(dt)
        torch.cuda.synchronize()
        G = oracle_grid(O, dd)
        O.fill_periodic(G)
        prm = O.params()
        assert float(dt.item()) == O.cfl_dt(G, prm)
        out = from_device(patch)
        for f in FIELDS:
            assert np.array_equal(out[f], getattr(G, f)), f
        # a second call starts from a cleared maximum
        plan.ppm_cfl_dt(dt)
        torch.cuda.synchronize()
        assert float(dt.item()) == O.cfl_dt(G, prm)
        plan.close()


def test_uniform_state_preserved_on_gpu(P):
    import torch
    d = W.uniform_grid(16, 8, 12, 1.0, (0.5, -0.25, 0.125), 0.5)
    patch = to_device(d, P.PPM_FP64)
    plan = P.Plan([patch], 1, P.PPM_FP64, P.params())
    dt = _dt_tensor()
    dt.fill_(0.01)
    for s in range(3):
        plan.ppm_step(dt, s % 2)
    torch.cuda.synchronize()
    out = from_device(patch)
    for f in FIELDS:
        assert np.array_equal(out[f], d[f]), f
    plan.close()


def test_sweep_extents_on_gpu(P, O):
    import torch
    d = W.random_grid(7, 6, 5, 3, W.GENTLE, seeded_ghosts=True)
    for axis in range(3):
        for mask in range(8):
            mask &= ~(1 << axis)
            patch = to_device(d, P.PPM_FP64)
            plan = P.Plan([patch], 1, P.PPM_FP64, P.params())
            dt = _dt_tensor()
            dt.fill_(1e-3)
            plan.ppm_sweep(dt, axis, mask)
            torch.cuda.synchronize()
            out = from_device(patch)
            G = oracle_grid(O, d)
            O.sweep(G, O.params(), 1e-3, axis, mask)
            for f in FIELDS:
                assert np.array_equal(out[f], getattr(G, f)) or \
                    np.max(np.abs(out[f] - getattr(G, f))) <= TOL64 * np.abs(getattr(G, f)).max()
            plan.close()


@pytest.mark.parametrize("tiles", ["lanes=0", "lanes=0 split=0", "lanes=7", "lanes=7 lanes_block=64",
                                   "block=64", "lanes=0 block=64 tail_round=640",
                                   "lanes=0 split=0 block=64 tail_round=640",
                                   "block=128 lanes_block=64 tail_round=1024"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_both_sweep_kernels_on_every_axis(P, O, tiles, prec):
    # The pencil-marching kernel and the lane-parallel kernel must agree with
    # the oracle along every axis, on grids long enough for several 54-cell
    # lane segments and with ragged tails; tail_round: each marching sweep
    # marches whole rounds of pencils and streams the rest one per wave.
    # These grids have few pencils, so marching sweeps run two threads per
    # pencil unless split=0.
    d = W.random_grid(131, 37, 61, 31337, W.SHOCKED)
    pr = P.PPM_FP64 if prec == "fp64" else P.PPM_MIXED
    d = stored_inputs(d, pr)
    g, gdt, gcnt, _ = _run_gpu_steps(P, d, 2, pr, tiles=tiles)
    o, odt, ocnt, _ = _run_oracle_steps(O, d, 2)
    if prec == "fp64":
        assert gdt == odt
        worst, differ = compare_fields(g, o, TOL64)
        print(f"{tiles}: worst {worst:.2e}, not bitwise {differ}, counts {gcnt} {ocnt}")
        assert gcnt == ocnt
    else:
        sl = (slice(3, -3),) * 3
        for f in FIELDS:
            l1 = np.abs(g[f][sl] - o[f][sl]).sum() / np.abs(o[f][sl]).sum()
            assert l1 <= 1e-5, (f, l1)


@pytest.mark.parametrize("ghost", [3, 4, 5, 6])
@pytest.mark.parametrize("tiles", ["lanes=0", "lanes=0 split=0"])
def test_split_marching_every_ghost_width(P, O, ghost, tiles):
    # Shocked input with flux registers, marching sweeps along every axis:
    # with split=1 (the default for so few pencils) each pencil is marched by
    # two threads, the second from max(5, ghost) cells before its first own
    # cell; results, counts and registers must equal the oracle's.
    d = W.random_grid(40, 24, 20, 4400 + ghost, W.SHOCKED, ghost=ghost)
    g, gdt, gcnt, greg = _run_gpu_steps(P, d, 2, P.PPM_FP64, ghost=ghost, with_reg=True,
                                        tiles=tiles)
    o, odt, ocnt, oreg = _run_oracle_steps(O, d, 2, ghost=ghost, with_reg=True)
    assert gdt == odt
    worst, differ = compare_fields(g, o, TOL64)
    print(f"ghost {ghost} {tiles}: worst {worst:.2e}, not bitwise {differ}, counts {gcnt}")
    assert differ == 0
    assert gcnt == ocnt
    assert np.array_equal(greg, oreg)


def test_full_size_512_step_in_bench_configuration(P, O):
    # The benchmark's workload (512^3, strongly shocked, seed 1002) and launch
    # configuration (default tiles: lane-parallel x sweeps, marching y and z),
    # one full step from the same stored input: FP64 compared with the oracle
    # cell by cell, mixed precision by per-field relative L1.
    import torch
    from paper_1307_2265_amd import autotune
    n = 512
    cfg = W.WORKLOADS["shocked512"]
    print("generating 512^3 input", flush=True)
    d = stored_inputs(W.random_grid(n, n, n, cfg["seed"], cfg["recipe"]), P.PPM_MIXED)
    print("oracle step", flush=True)
    G = oracle_grid(O, d)
    prm = O.params()
    O.fill_periodic(G)
    dt_ref = O.cfl_dt(G, prm)
    ocnt = O.step(G, prm, dt_ref, 0)
    sl = (slice(3, -3),) * 3
    for prec in (P.PPM_FP64, P.PPM_MIXED):
        print(f"gpu step, precision {prec}", flush=True)
        patch = to_device(d, prec)
        name = "fp64" if prec == P.PPM_FP64 else "mixed"
        plan = P.Plan([patch], 1, prec, P.params(), tile_config=autotune.best_tiles(f"single/{name}"))
        dt = _dt_tensor()
        plan.ppm_fill_periodic()
        plan.ppm_cfl_dt(dt)
        plan.ppm_step(dt, 0)
        torch.cuda.synchronize()
        assert float(dt.item()) == dt_ref
        counts = plan.ppm_event_counts()
        for f in FIELDS:
            a = getattr(patch, f)[3:-3, 3:-3, 3:-3].double().cpu().numpy()
            b = getattr(G, f)[sl]
            if prec == P.PPM_FP64:
                differ = int(np.count_nonzero(a != b))
                scale = np.maximum(np.abs(b), np.abs(b).mean())
                worst = float(np.max(np.abs(a - b) / scale))
                print(f"fp64 {f}: worst {worst:.2e}, cells not bitwise equal {differ}")
                assert worst <= TOL64
            else:
                l1 = float(np.abs(a - b).sum() / np.abs(b).sum())
                print(f"mixed {f}: relative L1 {l1:.2e}")
                assert l1 <= 1e-5
            del a
        if prec == P.PPM_FP64:
            assert counts == (ocnt.fallback_faces, ocnt.floored_cells)
        plan.close()
        del patch
        torch.cuda.empty_cache()


def test_config1_256_ten_steps_fp64(P, O):
    # The 256^3 workload (gentle white noise, seed 1001): ten steps with the
    # device CFL dt each step, in the single-grid launch configuration of the
    # benchmark, against ten oracle steps with the oracle's own dt.
    from paper_1307_2265_amd import autotune
    cfg = W.WORKLOADS["gentle256"]
    n = cfg["n"]
    print("generating 256^3 input", flush=True)
    d = W.random_grid(n, n, n, cfg["seed"], cfg["recipe"])
    g, dg, cg, _ = _run_gpu_steps(P, d, cfg["steps"], P.PPM_FP64,
                                  tiles=autotune.best_tiles("single/fp64"))
    print("oracle steps", flush=True)
    o, do, co, _ = _run_oracle_steps(O, d, cfg["steps"])
    assert dg == do
    worst, differ = compare_fields(g, o, TOL64, region=(slice(3, -3),) * 3)
    print(f"256^3 x 10 steps: worst {worst:.2e}, cells not bitwise equal {differ}, "
          f"counts {cg} {co}")
    assert cg == co


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_config3_full_batch_in_bench_configuration(P, O, prec):
    # The full 4096-patch batch (seed 1003) exactly as the benchmark runs it:
    # flat field buffers, autotuned launch shapes, one captured graph per step
    # (the three sweeps and the next step's dt, xyz then zyx; the first dt
    # from a CFL reduction), registers on.  Two steps; the oracle advances
    # every patch with its level's dt from its own CFL reduction.
    import torch
    from paper_1307_2265_amd import autotune
    from paper_1307_2265_amd import harness as H
    print("generating 4096 patches", flush=True)
    specs, fields = H.batch_input(4096)
    pr = P.PPM_FP64 if prec == "fp64" else P.PPM_MIXED
    run = H.Run.batch(specs, fields, pr, autotune.best_tiles(f"batch/{prec}"))
    run.make_graphs()
    run.ensure_dt()
    dts_g = []
    for s in range(2):
        torch.cuda.synchronize()
        dts_g.append(run.dt.cpu().numpy().copy())  # the dt step s advances with
        run.graphs[s].ppm_graph_launch()
    torch.cuda.synchronize()
    counts_g = run.plan.ppm_event_counts()
    print("oracle", flush=True)
    prm = O.params()
    nlev = run.nlevels
    grids = [oracle_grid(O, stored_inputs(f, pr), dx=(sp.dx,) * 3, with_reg=True)
             for f, sp in zip(fields, specs)]
    counts_o = [0, 0]
    for s in range(2):
        smax = np.zeros(nlev)
        for G, sp in zip(grids, specs):
            smax[sp.level] = max(smax[sp.level], O.cfl_signal_max(G, prm))
        dto = np.where(smax > 0, prm.cfl / np.where(smax > 0, smax, 1.0), np.inf)
        if prec == "fp64":
            assert np.array_equal(dts_g[s], dto), (s, dts_g[s], dto)
        else:
            assert np.allclose(dts_g[s], dto, rtol=1e-5), (s, dts_g[s], dto)
        for G, sp in zip(grids, specs):
            c = O.step(G, prm, float(dts_g[s][sp.level] if prec == "mixed" else dto[sp.level]),
                       s)
            counts_o[0] += c.fallback_faces
            counts_o[1] += c.floored_cells
    num = {f: 0.0 for f in FIELDS}
    den = {f: 0.0 for f in FIELDS}
    differ, worst = 0, 0.0
    sl = (slice(3, -3),) * 3
    for i, (p, G) in enumerate(zip(run.patches, grids)):
        g = from_device(p)
        if prec == "fp64":
            w, d = compare_fields({f: g[f][sl] for f in FIELDS},
                                  {f: getattr(G, f)[sl] for f in FIELDS}, TOL64)
            worst, differ = max(worst, w), differ + d
            reg = p.flux_reg.cpu().numpy()
            scale = np.maximum(np.abs(G.flux_reg), np.abs(G.flux_reg).mean())
            assert np.max(np.abs(reg - G.flux_reg) / scale) <= TOL64, i
        else:
            for f in FIELDS:
                num[f] += np.abs(g[f][sl] - getattr(G, f)[sl]).sum()
                den[f] += np.abs(getattr(G, f)[sl]).sum()
    run.close()
    if prec == "fp64":
        print(f"4096 patches x 2 steps: worst {worst:.2e}, cells not bitwise equal {differ}, "
              f"counts {counts_g} {tuple(counts_o)}")
        assert counts_g == tuple(counts_o)
    else:
        for f in FIELDS:
            print(f"4096 patches mixed, {f}: relative L1 after 2 steps {num[f] / den[f]:.2e}")
            assert num[f] / den[f] <= 1e-5


def _batch(P, O, npatch, seed, prec, tiles=None, steps=1, flat=True, flags=None):
    """Run a batch of uneven patches on the GPU and patch by patch on the oracle.
    flat: patches as views into shared field arrays (the marching sweeps may
    then span patches), else one allocation per patch field."""
    import torch
    specs = W.patch_specs(npatch, seed)
    nlev = 7
    fields = [stored_inputs(W.patch_fields(sp), prec) for sp in specs]
    if flat:
        patches = to_device_flat(fields, prec, [(sp.dx,) * 3 for sp in specs],
                                 [sp.level for sp in specs], with_reg=True)
    else:
        patches = [to_device(f, prec, dx=(sp.dx,) * 3, level=sp.level, with_reg=True)
                   for f, sp in zip(fields, specs)]
    gprm = P.params() if flags is None else P.params(flags=flags)
    plan = P.Plan(patches, nlev, prec, gprm, tile_config=tiles)
    dt = _dt_tensor(nlev)
    prm = O.params() if flags is None else O.params(flags=flags)
    grids = [oracle_grid(O, f, dx=(sp.dx,) * 3, with_reg=True) for f, sp in zip(fields, specs)]
    ocnt = [0, 0]
    dts_g, dts_o = [], []
    for s in range(steps):
        plan.ppm_cfl_dt(dt)
        plan.ppm_step(dt, s % 2)
        torch.cuda.synchronize()
        dts_g.append(dt.cpu().numpy().copy())
        smax = np.zeros(nlev)
        for G, sp in zip(grids, specs):
            smax[sp.level] = max(smax[sp.level], O.cfl_signal_max(G, prm))
        dto = np.where(smax > 0, prm.cfl / np.where(smax > 0, smax, 1.0), np.inf)
        dts_o.append(dto)
        for G, sp in zip(grids, specs):
            c = O.step(G, prm, float(dto[sp.level]), s % 2)
            ocnt[0] += c.fallback_faces
            ocnt[1] += c.floored_cells
    gcnt = plan.ppm_event_counts()
    outs = [(from_device(p), p.flux_reg.cpu().numpy()) for p in patches]
    plan.close()
    return specs, outs, grids, dts_g, dts_o, gcnt, tuple(ocnt)


@pytest.mark.parametrize("tiles,flat", [(None, True), ("lanes=0", True), ("lanes=7", True),
                                        ("persistent=0", True), ("persistent=0 lanes=0", True),
                                        ("persistent=0 lanes=0 group=1 block=128", True),
                                        ("persistent=0 lanes=0", False),
                                        ("persistent=0 lanes=0 group=0", True),
                                        ("persistent=1 batch_block=64", True)])
def test_batch_of_uneven_patches_fp64(P, O, tiles, flat):
    specs, outs, grids, dg, do, gcnt, ocnt = _batch(P, O, 48, 1003, P.PPM_FP64, tiles, steps=2,
                                                    flat=flat)
    for a, b in zip(dg, do):
        assert np.array_equal(a, b), (a, b)
    differ = 0
    for (g, greg), G in zip(outs, grids):
        sl = (slice(3, -3),) * 3
        _, d = compare_fields({f: g[f][sl] for f in FIELDS},
                              {f: getattr(G, f)[sl] for f in FIELDS}, TOL64)
        differ += d
        scale = np.maximum(np.abs(G.flux_reg), np.abs(G.flux_reg).mean())
        assert np.max(np.abs(greg - G.flux_reg) / scale) <= TOL64
    print(f"{tiles} (flat {flat}): 48 patches, active cells not bitwise equal: {differ}, "
          f"counts {gcnt} {ocnt}")
    assert gcnt == ocnt


@pytest.mark.parametrize("tiles", [None, "persistent=0 lanes=0"])
def test_batch_of_uneven_patches_mixed(P, O, tiles):
    specs, outs, grids, dg, do, _, _ = _batch(P, O, 32, 2003, P.PPM_MIXED, tiles)
    num = {f: 0.0 for f in FIELDS}
    den = {f: 0.0 for f in FIELDS}
    for (g, _), G in zip(outs, grids):
        sl = (slice(3, -3),) * 3
        for f in FIELDS:
            num[f] += np.abs(g[f][sl] - getattr(G, f)[sl]).sum()
            den[f] += np.abs(getattr(G, f)[sl]).sum()
    for f in FIELDS:
        print(f"batch mixed {f}: relative L1 {num[f] / den[f]:.2e}")
        assert num[f] / den[f] <= 1e-5


@pytest.mark.parametrize("batch,fused", [(False, False), (True, False), (False, True),
                                         (True, True)])
def test_graph_replays_match_eager_steps(P, O, batch, fused):
    # Capture fill (single grid) + CFL + step -- or fill + step with the next
    # dt (fused) -- into a HIP graph, replay it several times with eager work
    # and synchronisations in between, and check every replay against the
    # same steps run eagerly.
    import torch
    step = P.PPM_GRAPH_STEP_CFL if fused else P.PPM_GRAPH_CFL | P.PPM_GRAPH_STEP
    if batch:
        specs = W.patch_specs(24, 77)
        fields = [W.patch_fields(sp) for sp in specs]
        mk = lambda: [to_device(f, P.PPM_FP64, dx=(sp.dx,) * 3, level=sp.level)
                      for f, sp in zip(fields, specs)]
        nlev, parts = 7, step
    else:
        d = W.random_grid(40, 24, 16, 5, W.SHOCKED)
        mk = lambda: [to_device(d, P.PPM_FP64)]
        nlev, parts = 1, P.PPM_GRAPH_FILL | step
    A, B = mk(), mk()
    pa = P.Plan(A, nlev, P.PPM_FP64, P.params())
    pb = P.Plan(B, nlev, P.PPM_FP64, P.params())
    dta, dtb = _dt_tensor(nlev), _dt_tensor(nlev)
    graphs = [P.Graph(pb, dtb, order, parts) for order in (0, 1)]
    if fused:  # the first step's dt comes from a plain reduction
        if not batch:
            pb.ppm_fill_periodic()
        pb.ppm_cfl_dt(dtb)
    for s in range(4):
        if not batch:
            pa.ppm_fill_periodic()
        pa.ppm_cfl_dt(dta)
        if fused:
            torch.cuda.synchronize()
            assert torch.equal(dta, dtb)
        pa.ppm_step(dta, s % 2)
        graphs[s % 2].ppm_graph_launch()
        torch.cuda.synchronize()
        junk = torch.ones(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        if not fused:
            assert torch.equal(dta, dtb)
        for pA, pB in zip(A, B):
            for f in FIELDS:
                assert torch.equal(getattr(pA, f), getattr(pB, f)), (s, f)
    del junk
    for g in graphs:
        g.close()
    pa.close()
    pb.close()


@pytest.mark.parametrize("case", ["single-fp64", "single-mixed", "single-lanes7", "single-tail",
                                  "batch-fp64", "batch-mixed", "batch-persistent", "batch-march",
                                  "batch-march-ungrouped"])
def test_step_with_next_dt_equals_step_then_cfl(P, case):
    # ppm_step_cfl takes the next step's CFL timestep from the values its last
    # sweep stores; it must leave the same fields as ppm_step and the same dt
    # as a separate ppm_cfl_dt, bit for bit, step after step (both orders).
    import torch
    prec = P.PPM_MIXED if "mixed" in case else P.PPM_FP64
    tiles = {"single-lanes7": "lanes=7", "single-tail": "block=64 lanes_block=64 tail_round=320",
             "batch-persistent": "persistent=1",
             "batch-march": "persistent=0 lanes=0",
             "batch-march-ungrouped": "persistent=0 lanes=0 group=0"}.get(case)
    if case.startswith("single"):
        d = W.random_grid(40, 28, 20, 11, W.SHOCKED)
        mk = lambda: [to_device(stored_inputs(d, prec), prec)]
        nlev, periodic = 1, True
    else:
        specs = W.patch_specs(40, 21)
        fields = [stored_inputs(W.patch_fields(sp), prec) for sp in specs]
        mk = lambda: to_device_flat(fields, prec, [(sp.dx,) * 3 for sp in specs],
                                    [sp.level for sp in specs], with_reg=True)
        nlev, periodic = 7, False
    A, B = mk(), mk()
    pa = P.Plan(A, nlev, prec, P.params(), tile_config=tiles)
    pb = P.Plan(B, nlev, prec, P.params(), tile_config=tiles)
    dta, dtb = _dt_tensor(nlev), _dt_tensor(nlev)
    if periodic:
        pb.ppm_fill_periodic()
    pb.ppm_cfl_dt(dtb)
    for s in range(4):
        if periodic:
            pa.ppm_fill_periodic()
            pb.ppm_fill_periodic()
        pa.ppm_cfl_dt(dta)
        assert torch.equal(dta, dtb), (s, dta, dtb)
        pa.ppm_step(dta, s % 2)
        pb.ppm_step_cfl(dtb, s % 2)
        torch.cuda.synchronize()
        for pA, pB in zip(A, B):
            for f in FIELDS:
                assert torch.equal(getattr(pA, f), getattr(pB, f)), (s, f)
            if pA.flux_reg is not None:
                assert torch.equal(pA.flux_reg, pB.flux_reg), s
    if periodic:
        pa.ppm_fill_periodic()
    pa.ppm_cfl_dt(dta)
    torch.cuda.synchronize()
    assert torch.equal(dta, dtb)
    assert pa.ppm_event_counts() == pb.ppm_event_counts()
    pa.close()
    pb.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sweeps_with_cfl_finalize_equal_fused_step(P, prec):
    # ppm_sweep, ppm_sweep, ppm_sweep_cfl + ppm_cfl_finalize (the form the
    # benchmark times sweep by sweep) against ppm_step_cfl: same fields, same
    # next dt, both sweep orders.
    import torch
    pr = P.PPM_FP64 if prec == "fp64" else P.PPM_MIXED
    d = stored_inputs(W.random_grid(36, 30, 22, 17, W.SHOCKED), pr)
    A, B = [to_device(d, pr)], [to_device(d, pr)]
    pa = P.Plan(A, 1, pr, P.params())
    pb = P.Plan(B, 1, pr, P.params())
    dta, dtb = _dt_tensor(), _dt_tensor()
    for p_, dt in ((pa, dta), (pb, dtb)):
        p_.ppm_fill_periodic()
        p_.ppm_cfl_dt(dt)
    orders = ((0, 1, 2), (2, 1, 0))
    for s in range(4):
        pa.ppm_fill_periodic()
        pb.ppm_fill_periodic()
        mask = 0
        for k, axis in enumerate(orders[s % 2]):
            if k < 2:
                pa.ppm_sweep(dta, axis, mask)
            else:
                pa.ppm_sweep_cfl(dta, axis, mask)
            mask |= 1 << axis
        pa.ppm_cfl_finalize(dta)
        pb.ppm_step_cfl(dtb, s % 2)
        torch.cuda.synchronize()
        assert torch.equal(dta, dtb), s
        for f in FIELDS:
            assert torch.equal(getattr(A[0], f), getattr(B[0], f)), (s, f)
    pa.close()
    pb.close()
