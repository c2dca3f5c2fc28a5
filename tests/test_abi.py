"""The C ABI library: it loads, exports every function include/ppm.h declares,
and rejects invalid arguments before touching the GPU (CPU only)."""
import ctypes as C
import os
import re

import pytest

from paper_1307_2265_amd import ppm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "ppm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ppm_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    names = _declared_functions()
    assert "ppm_step" in names and "ppm_cfl_dt" in names and len(names) >= 10
    L = C.CDLL(ppm.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(ppm.SIGNATURES), set(names) ^ set(ppm.SIGNATURES)


def test_status_strings_and_reg_size():
    L = ppm.lib()
    assert L.ppm_status_str(ppm.PPM_EINVAL).startswith(b"PPM_EINVAL")
    assert ppm.ppm_flux_reg_size(4, 5, 6) == 12 * (5 * 6 + 4 * 6 + 4 * 5)


def _patch(**kw):
    base = dict(nx=8, ny=8, nz=8, ghost=3, level=0, bc=0, dx=0.1, dy=0.1, dz=0.1,
                rho=1, vx=1, vy=1, vz=1, etot=1, eint=1, flux_reg=None)
    base.update(kw)
    return ppm.ppm_patch(**base)


@pytest.mark.parametrize("patch_kw,prm_kw,msg", [
    (dict(ghost=2), {}, "ghost"),
    (dict(nx=0), {}, "dims"),
    (dict(level=3), {}, "level"),
    (dict(dx=0.0), {}, "cell widths"),
    (dict(rho=None), {}, "NULL field"),
    (dict(bc=2), {}, "bc must be"),
    ({}, dict(gamma=1.0), "gamma"),
    ({}, dict(cfl=1.5), "cfl"),
    ({}, dict(riemann_max_iter=0), "riemann_max_iter"),
    ({}, dict(rho_floor=1e-120), "floor"),    # below the fast division's range bound
    ({}, dict(p_floor=0.0), "floor"),
    ({}, dict(e_floor=0.0), "floor"),
    ({}, dict(flags=99), "flag"),
    ({}, dict(flags=0x80000000), "flag"),     # library-internal bit
    (dict(gx=1, gy=1), {}, "acceleration"),   # gz missing
])
def test_plan_create_rejects_invalid_arguments(patch_kw, prm_kw, msg):
    L = ppm.lib()
    arr = (ppm.ppm_patch * 1)(_patch(**patch_kw))
    prm = ppm.params(**prm_kw)
    h = C.c_void_p()
    st = L.ppm_plan_create(C.byref(h), arr, 1, 2, ppm.PPM_FP64, C.byref(prm), None, None)
    assert st == ppm.PPM_EINVAL
    assert not h.value
    assert msg in L.ppm_last_error().decode()


@pytest.mark.parametrize("prm_kw", [dict(rho_floor=1e-40), dict(p_floor=1e-45),
                                    dict(rho_floor=1e-60, p_floor=1e-60), dict(p_floor=1e39)])
def test_mixed_precision_rejects_floors_outside_the_normal_float_range(prm_kw):
    # PPM_MIXED stores the density in float: a floor below FLT_MIN would be
    # stored as a subnormal or zero, and the next sweep would divide by it
    L = ppm.lib()
    arr = (ppm.ppm_patch * 1)(_patch())
    prm = ppm.params(**prm_kw)
    h = C.c_void_p()
    st = L.ppm_plan_create(C.byref(h), arr, 1, 1, ppm.PPM_MIXED, C.byref(prm), None, None)
    assert st == ppm.PPM_EINVAL and not h.value
    assert "normal float range" in L.ppm_last_error().decode()
    # the same floors are valid in FP64 (checked up to the first device call)
    st = L.ppm_plan_create(C.byref(h), arr, 1, 1, ppm.PPM_FP64, C.byref(prm), b"warp=1", None)
    assert st == ppm.PPM_EINVAL and "unknown key" in L.ppm_last_error().decode()


def test_calls_on_null_plan_are_rejected():
    L = ppm.lib()
    assert L.ppm_step(None, None, 0, None) == ppm.PPM_EINVAL
    assert L.ppm_cfl_dt(None, None, None) == ppm.PPM_EINVAL
    assert L.ppm_fill_periodic(None, None) == ppm.PPM_EINVAL
    assert L.ppm_sweep(None, None, 0, 0, None) == ppm.PPM_EINVAL
    assert L.ppm_step_cfl(None, None, 0, None) == ppm.PPM_EINVAL
    assert L.ppm_sweep_cfl(None, None, 0, 0, None) == ppm.PPM_EINVAL
    assert L.ppm_cfl_finalize(None, None, None) == ppm.PPM_EINVAL
    assert L.ppm_fill_boundary(None, 0, None, None, None) == ppm.PPM_EINVAL
    assert L.ppm_set_hierarchy(None, None, None) == ppm.PPM_EINVAL
    assert L.ppm_fill_ghosts(None, 0, None) == ppm.PPM_EINVAL
    assert L.ppm_event_counts(None, None, None, 0, None) == ppm.PPM_EINVAL
    assert L.ppm_set_expansion(None, None) == ppm.PPM_EINVAL
    assert L.ppm_amr_step(None, None) == ppm.PPM_EINVAL
    assert L.ppm_amr_set_expansion(None, None) == ppm.PPM_EINVAL
    assert L.ppm_amr_times(None, None, None) == ppm.PPM_EINVAL
    assert L.ppm_amr_step_log(None, None, None, 0, None) == ppm.PPM_EINVAL
    assert L.ppm_amr_event_counts(None, None, None, None) == ppm.PPM_EINVAL
    assert L.ppm_amr_destroy(None) == ppm.PPM_OK
    assert L.ppm_expansion(None, None, None) == ppm.PPM_EINVAL
    assert L.ppm_plan_destroy(None) == ppm.PPM_OK
    assert L.ppm_fp64_ops(None, None, None, None, 1, None) == ppm.PPM_EINVAL


def test_bad_tile_config_is_rejected():
    L = ppm.lib()
    arr = (ppm.ppm_patch * 1)(_patch())
    prm = ppm.params()
    h = C.c_void_p()
    st = L.ppm_plan_create(C.byref(h), arr, 1, 1, ppm.PPM_FP64, C.byref(prm), b"block=100",
                           None)
    assert st == ppm.PPM_EINVAL and "block" in L.ppm_last_error().decode()
    st = L.ppm_plan_create(C.byref(h), arr, 1, 1, ppm.PPM_FP64, C.byref(prm), b"warp=3", None)
    assert st == ppm.PPM_EINVAL and "unknown key" in L.ppm_last_error().decode()
    st = L.ppm_plan_create(C.byref(h), arr, 1, 1, ppm.PPM_FP64, C.byref(prm), b"tail=2", None)
    assert st == ppm.PPM_EINVAL and "tail" in L.ppm_last_error().decode()
    st = L.ppm_plan_create(C.byref(h), arr, 1, 1, ppm.PPM_FP64, C.byref(prm), b"split=2", None)
    assert st == ppm.PPM_EINVAL and "split" in L.ppm_last_error().decode()
    st = L.ppm_plan_create(C.byref(h), arr, 1, 1, ppm.PPM_FP64, C.byref(prm),
                           b"block=128 tail_round=320", None)
    assert st == ppm.PPM_EINVAL and "multiple of block" in L.ppm_last_error().decode()
    assert not h.value


def test_persistent_launch_rejects_patches_too_large_for_one_workgroup():
    # a workgroup of the persistent launch owns a whole patch; 2^21 active
    # cells is the limit (the check runs before anything touches the device)
    L = ppm.lib()
    arr = (ppm.ppm_patch * 2)(_patch(), _patch(nx=128, ny=128, nz=129))
    prm = ppm.params()
    h = C.c_void_p()
    st = L.ppm_plan_create(C.byref(h), arr, 2, 1, ppm.PPM_FP64, C.byref(prm), b"persistent=1",
                           None)
    assert st == ppm.PPM_EINVAL and "persistent=1" in L.ppm_last_error().decode()
    assert not h.value


def test_grouping_needs_patches_in_shared_arrays():
    # explicit group=1 with patches whose fields are separate allocations
    L = ppm.lib()
    arr = (ppm.ppm_patch * 2)(_patch(), _patch(rho=1024, vx=2048, vy=4096, vz=8192, etot=16384,
                                               eint=32768))
    prm = ppm.params()
    h = C.c_void_p()
    st = L.ppm_plan_create(C.byref(h), arr, 2, 1, ppm.PPM_FP64, C.byref(prm),
                           b"group=1 persistent=0", None)
    assert st == ppm.PPM_EINVAL and "group=1" in L.ppm_last_error().decode()
    assert not h.value


def _amr_patch(level, dims, reg=True, bc=0):
    return _patch(nx=dims[0], ny=dims[1], nz=dims[2], level=level, bc=bc,
                  flux_reg=1 if (reg and level > 0) else None)


@pytest.mark.parametrize("spec,msg", [
    ([(0, -1, (0, 0, 0), (16, 16, 16)), (0, -1, (0, 0, 0), (16, 16, 16))], "exactly one root"),
    ([(0, -1, (0, 0, 0), (16, 16, 16)), (1, 0, (8, 8, 8), (12, 12, 12), False)], "flux registers"),
    ([(0, -1, (0, 0, 0), (16, 16, 16)), (1, 0, (9, 8, 8), (12, 12, 12))], "cell boundaries"),
    ([(0, -1, (0, 0, 0), (16, 16, 16)), (1, 0, (0, 8, 8), (12, 12, 12))], "inside the parent"),
    ([(0, -1, (0, 0, 0), (16, 16, 16)), (1, 0, (8, 8, 8), (12, 12, 12)),
      (1, 0, (12, 12, 12), (8, 8, 8))], "overlap"),
    ([(0, -1, (0, 0, 0), (16, 16, 16), True, 1)], "PPM_BC_PERIODIC"),
])
def test_amr_create_rejects_invalid_hierarchies(spec, msg):
    # validation happens before any device call
    L = ppm.lib()
    pts, pls = [], []
    for s in spec:
        lev, par, start, dims = s[:4]
        reg = s[4] if len(s) > 4 else True
        bc = s[5] if len(s) > 5 else 0
        pts.append(_amr_patch(lev, dims, reg, bc))
        pl = ppm.ppm_patch_place()
        pl.parent, pl.refine = par, 2
        for a in range(3):
            pl.start[a] = start[a]
        pls.append(pl)
    arr = (ppm.ppm_patch * len(pts))(*pts)
    parr = (ppm.ppm_patch_place * len(pls))(*pls)
    prm = ppm.params()
    h = C.c_void_p()
    st = L.ppm_amr_create(C.byref(h), arr, parr, len(pts), 3, ppm.PPM_FP64, C.byref(prm), None,
                          None, None)
    assert st == ppm.PPM_EINVAL
    assert not h.value
    assert msg in L.ppm_last_error().decode()
