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
                           to_device)

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


@pytest.mark.parametrize("tiles", [None, "lanes=0", "lanes=7"])
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


@pytest.mark.parametrize("tiles", ["lanes=0", "lanes=7", "lanes=7 lanes_block=64",
                                   "block=64"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_both_sweep_kernels_on_every_axis(P, O, tiles, prec):
    # The pencil-marching kernel and the lane-parallel kernel must agree with
    # the oracle along every axis, on grids long enough for several 54-cell
    # lane segments and with ragged tails.
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
