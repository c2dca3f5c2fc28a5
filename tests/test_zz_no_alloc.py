"""ppm_step_cfl_noalloc, the step that allocates nothing, against the plan
path it stands in for (GPU): fill, CFL and step of a plan (ppm_fill_periodic,
ppm_cfl_dt, ppm_step_cfl) and the no-alloc call with both parts must leave
identical fields, timesteps and event counts, over two calls in a row whose
second has a smaller input (so nothing of the first call's scratch contents
may leak into the second), in both precisions, for one patch and for several
patches of different levels."""
import numpy as np
import pytest

from paper_1307_2265_amd import workloads as W
from tests.helpers import FIELDS, from_device, stored_inputs, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    from paper_1307_2265_amd import ppm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ppm.lib()
    return ppm


def _patches(P, pr, dims_list, seed, levels=None):
    out = []
    for i, dims in enumerate(dims_list):
        d = stored_inputs(W.random_grid(*dims, seed + i, W.SHOCKED), pr)
        lev = 0 if levels is None else levels[i]
        dx = 2.0 ** -lev / max(dims)
        out.append(to_device(d, pr, dx=(dx, dx, dx), level=lev, with_reg=True))
    return out


def _clone(P, patches):
    import torch
    out = []
    for p in patches:
        t = {f: getattr(p, f).clone() for f in FIELDS}
        out.append(P.Patch(**t, dx=p.dx, dy=p.dy, dz=p.dz, ghost=p.ghost, level=p.level,
                           flux_reg=torch.zeros_like(p.flux_reg)))
    return out


def _compare(a_list, b_list):
    for i, (a, b) in enumerate(zip(a_list, b_list)):
        ga, gb = from_device(a), from_device(b)
        for f in FIELDS:
            assert np.array_equal(ga[f], gb[f]), (i, f)
        assert np.array_equal(a.flux_reg.cpu().numpy(), b.flux_reg.cpu().numpy()), i


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["one-patch", "several-patches"])
def test_noalloc_step_equals_the_plan_path(P, prec, case):
    import torch
    pr = P.PPM_FP64 if prec == "fp64" else P.PPM_MIXED
    if case == "one-patch":
        calls = [([(40, 36, 28)], None, 1), ([(12, 10, 8)], None, 1)]
    else:
        calls = [([(24, 16, 20), (16, 16, 16), (8, 12, 24)], [0, 1, 2], 3),
                 ([(8, 8, 12), (12, 8, 8)], [1, 0], 2)]
    prm = P.params()
    for c, (dims, levels, nlev) in enumerate(calls):
        print(f"{prec} {case} call {c}: dims {dims} levels {levels}", flush=True)
        ref = _patches(P, pr, dims, 7100 + 10 * c, levels)
        mine = _clone(P, ref)
        # the plan path
        plan = P.Plan(ref, nlev, pr, prm)
        dt_ref = torch.zeros(nlev, dtype=torch.float64, device="cuda")
        plan.ppm_event_counts(reset=True)
        plan.ppm_fill_periodic()
        plan.ppm_cfl_dt(dt_ref)
        plan.ppm_step_cfl(dt_ref, c % 2)
        ev_ref = plan.ppm_event_counts()
        # no plan, no allocation
        dt = torch.full((nlev,), -1.0, dtype=torch.float64, device="cuda")
        ev = P.ppm_step_cfl_noalloc(mine, nlev, pr, prm, dt, c % 2,
                                    P.PPM_NOALLOC_FILL | P.PPM_NOALLOC_CFL, events=True)
        torch.cuda.synchronize()
        assert ev == ev_ref, (ev, ev_ref)
        assert np.array_equal(dt.cpu().numpy(), dt_ref.cpu().numpy())
        _compare(mine, ref)
        # a second step from the timestep it returned (no CFL part)
        plan.ppm_fill_periodic()
        plan.ppm_step_cfl(dt_ref, 1 - c % 2)
        P.ppm_step_cfl_noalloc(mine, nlev, pr, prm, dt, 1 - c % 2, P.PPM_NOALLOC_FILL)
        torch.cuda.synchronize()
        assert np.array_equal(dt.cpu().numpy(), dt_ref.cpu().numpy())
        _compare(mine, ref)
        plan.close()


def test_noalloc_rejects_sizes_beyond_its_scratch(P):
    import ctypes as C
    import torch
    pr = P.PPM_FP64
    ps = _patches(P, pr, [(8, 8, 8)], 7300)
    arr = (P.ppm_patch * 17)(*([ps[0].to_c()] * 17))
    dt = torch.zeros(17, dtype=torch.float64, device="cuda")
    prm = P.params()
    L = P.lib()
    st = L.ppm_step_cfl_noalloc(arr, 17, 1, pr, C.byref(prm), dt.data_ptr(), 0, 0, None, None)
    assert st == P.PPM_EINVAL and "1..16" in L.ppm_last_error().decode()
    st = L.ppm_step_cfl_noalloc(arr, 1, 17, pr, C.byref(prm), dt.data_ptr(), 0, 0, None, None)
    assert st == P.PPM_EINVAL and "1..16" in L.ppm_last_error().decode()
