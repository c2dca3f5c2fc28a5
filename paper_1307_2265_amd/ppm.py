"""Thin Python binding of libppm.so (include/ppm.h).

Argument marshalling only: every function below forwards to the C ABI of the
same name, and every step of the PPM update runs in the HIP kernels of that
library.  PyTorch supplies device memory and streams.  There is no fallback:
if the library is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libppm.so")

PPM_OK, PPM_EINVAL, PPM_ENOMEM, PPM_EHIP, PPM_EUNSUPPORTED = 0, -1, -2, -3, -4
PPM_FP64, PPM_MIXED = 0, 1
PPM_STEEPEN, PPM_FLATTEN, PPM_DUAL_ENERGY, PPM_FALLBACK_HLL = 1, 2, 4, 8
PPM_ALL_FLAGS = 15
PPM_HLLC = 16  # HLLC face fluxes instead of two-shock
PPM_DIFFUSION = 32  # CW84's diffusive flux where the flow converges
ORDERS = {"xyz": 0, "zyx": 1, "xzy": 2, "yxz": 3, "yzx": 4, "zxy": 5}
PPM_GRAPH_FILL, PPM_GRAPH_CFL, PPM_GRAPH_STEP, PPM_GRAPH_STEP_CFL = 1, 2, 4, 8
PPM_BC_PERIODIC, PPM_BC_SUPPLIED = 0, 1
PPM_FACE_PERIODIC, PPM_FACE_REFLECTING, PPM_FACE_OUTFLOW, PPM_FACE_INFLOW = 0, 1, 2, 3

# Every function the header declares, with (restype, argtypes).
_vp = C.c_void_p


class ppm_patch(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("ghost", C.c_int32),
                ("level", C.c_int32), ("bc", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("rho", _vp), ("vx", _vp), ("vy", _vp), ("vz", _vp),
                ("etot", _vp), ("eint", _vp), ("flux_reg", _vp),
                ("gx", _vp), ("gy", _vp), ("gz", _vp)]


class ppm_params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double), ("eta1", C.c_double),
                ("eta2", C.c_double), ("rho_floor", C.c_double), ("p_floor", C.c_double),
                ("e_floor", C.c_double), ("riemann_rtol", C.c_double),
                ("riemann_max_iter", C.c_int32), ("flags", C.c_uint32)]


class ppm_patch_place(C.Structure):
    _fields_ = [("parent", C.c_int32), ("refine", C.c_int32), ("start", C.c_int32 * 3)]


SIGNATURES = {
    "ppm_flux_reg_size": (C.c_int64, [C.c_int32, C.c_int32, C.c_int32]),
    "ppm_plan_create": (C.c_int, [C.POINTER(_vp), C.POINTER(ppm_patch), C.c_int32, C.c_int32,
                                  C.c_int, C.POINTER(ppm_params), C.c_char_p, _vp]),
    "ppm_plan_destroy": (C.c_int, [_vp]),
    "ppm_fill_periodic": (C.c_int, [_vp, _vp]),
    "ppm_set_hierarchy": (C.c_int, [_vp, C.POINTER(ppm_patch_place), _vp]),
    "ppm_fill_ghosts": (C.c_int, [_vp, C.c_int32, _vp]),
    "ppm_fill_boundary": (C.c_int, [_vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                    _vp]),
    "ppm_amr_create": (C.c_int, [C.POINTER(_vp), C.POINTER(ppm_patch),
                                 C.POINTER(ppm_patch_place), C.c_int32, C.c_int32, C.c_int,
                                 C.POINTER(ppm_params), C.POINTER(C.c_int32),
                                 C.POINTER(C.c_double), _vp]),
    "ppm_amr_destroy": (C.c_int, [_vp]),
    "ppm_amr_step": (C.c_int, [_vp, _vp]),
    "ppm_amr_set_expansion": (C.c_int, [_vp, _vp]),
    "ppm_amr_times": (C.c_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "ppm_amr_step_log": (C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_int32,
                                   C.POINTER(C.c_int32)]),
    "ppm_amr_event_counts": (C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), _vp]),
    "ppm_set_expansion": (C.c_int, [_vp, _vp]),
    "ppm_expansion": (C.c_int, [_vp, _vp, _vp]),
    "ppm_cfl_dt": (C.c_int, [_vp, _vp, _vp]),
    "ppm_step": (C.c_int, [_vp, _vp, C.c_int32, _vp]),
    "ppm_step_cfl": (C.c_int, [_vp, _vp, C.c_int32, _vp]),
    "ppm_sweep": (C.c_int, [_vp, _vp, C.c_int32, C.c_int32, _vp]),
    "ppm_sweep_cfl": (C.c_int, [_vp, _vp, C.c_int32, C.c_int32, _vp]),
    "ppm_cfl_finalize": (C.c_int, [_vp, _vp, _vp]),
    "ppm_event_counts": (C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_int32,
                                   _vp]),
    "ppm_graph_create": (C.c_int, [C.POINTER(_vp), _vp, _vp, C.c_int32, C.c_uint32, _vp]),
    "ppm_graph_launch": (C.c_int, [_vp, _vp]),
    "ppm_graph_destroy": (C.c_int, [_vp]),
    "ppm_fp64_ops": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int64, _vp]),
    "ppm_step_cfl_noalloc": (C.c_int, [C.POINTER(ppm_patch), C.c_int32, C.c_int32, C.c_int,
                                       C.POINTER(ppm_params), _vp, C.c_int32, C.c_uint32,
                                       C.POINTER(C.c_int64), _vp]),
    "ppm_status_str": (C.c_char_p, [C.c_int]),
    "ppm_last_error": (C.c_char_p, []),
}

_lib = None


class PPMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def lib():
    """Load libppm.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_1307_2265_amd/build.py` (no fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int, what: str):
    if status != PPM_OK:
        msg = lib().ppm_last_error().decode() or lib().ppm_status_str(status).decode()
        raise PPMError(status, f"{what}: {msg}")


def params(gamma=5.0 / 3.0, cfl=0.4, eta1=1e-3, eta2=0.1, rho_floor=1e-20, p_floor=1e-20,
           e_floor=1e-30, riemann_rtol=1e-13, riemann_max_iter=20,
           flags=PPM_ALL_FLAGS) -> ppm_params:
    return ppm_params(gamma, cfl, eta1, eta2, rho_floor, p_floor, e_floor, riemann_rtol,
                      riemann_max_iter, flags)


def ppm_flux_reg_size(nx: int, ny: int, nz: int) -> int:
    return int(lib().ppm_flux_reg_size(nx, ny, nz))


def ppm_fp64_ops(a, b, quot, root, stream=None) -> None:
    """quot = a / b and root = sqrt(a) by the library's FP64 division and
    square root (device float64 tensors of one length)."""
    n = a.numel()
    for t in (b, quot, root):
        assert t.numel() == n and t.is_contiguous()
    _check(lib().ppm_fp64_ops(a.data_ptr(), b.data_ptr(), quot.data_ptr(), root.data_ptr(), n,
                              _stream_handle(stream)), "ppm_fp64_ops")


PPM_NOALLOC_MAX_PATCHES = 16
PPM_NOALLOC_FILL, PPM_NOALLOC_CFL = 1, 2


def ppm_step_cfl_noalloc(patches: list, nlevels: int, precision: int, prm: ppm_params, dt,
                         sweep_order: int, parts: int = 0, events: bool = False, stream=None):
    """The C function of the same name: one step of up to 16 patches (and the
    next timestep in dt) without a plan and without allocating; with
    events=True returns (HLL faces, floored cells) of the step."""
    arr = (ppm_patch * len(patches))(*[p.to_c() for p in patches])
    ev = (C.c_int64 * 2)(0, 0)
    _check(lib().ppm_step_cfl_noalloc(arr, len(patches), nlevels, precision, C.byref(prm),
                                      dt.data_ptr(), sweep_order, parts, ev if events else None,
                                      _stream_handle(stream)), "ppm_step_cfl_noalloc")
    return (ev[0], ev[1]) if events else None


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream or None
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


@dataclass
class Patch:
    """One patch: six device tensors of shape (nz+2g, ny+2g, nx+2g).

    rho, vx, vy, vz are float64 (PPM_FP64) or float32 (PPM_MIXED); etot and
    eint are float64.  flux_reg is an optional float64 tensor of
    ppm_flux_reg_size(nx, ny, nz) elements.  bc: PPM_BC_PERIODIC (ghosts filled
    by ppm_fill_periodic) or PPM_BC_SUPPLIED (ghosts filled by the caller).
    accel: optional (gx, gy, gz), tensors of rho's dtype and shape, the
    gravitational acceleration at the cell centres (ghosts included).
    """
    rho: object
    vx: object
    vy: object
    vz: object
    etot: object
    eint: object
    dx: float
    dy: float
    dz: float
    ghost: int = 3
    level: int = 0
    flux_reg: object = None
    bc: int = PPM_BC_PERIODIC
    accel: tuple | None = None

    @property
    def dims(self):
        nz, ny, nx = self.rho.shape
        g = self.ghost
        return nx - 2 * g, ny - 2 * g, nz - 2 * g

    def fields(self):
        return [self.rho, self.vx, self.vy, self.vz, self.etot, self.eint]

    def to_c(self) -> ppm_patch:
        nx, ny, nz = self.dims
        shp = tuple(self.rho.shape)
        for t in self.fields():
            if tuple(t.shape) != shp or not t.is_contiguous() or t.device.type != "cuda":
                raise ValueError("patch fields must be contiguous CUDA tensors of one shape")
        acc = list(self.accel) if self.accel is not None else [None] * 3
        for t in acc:
            if t is not None and (tuple(t.shape) != shp or not t.is_contiguous()
                                  or t.dtype != self.rho.dtype or t.device.type != "cuda"):
                raise ValueError("accel must be contiguous CUDA tensors of rho's dtype and shape")
        ptr = lambda t: None if t is None else t.data_ptr()
        return ppm_patch(nx, ny, nz, self.ghost, self.level, self.bc, self.dx, self.dy, self.dz,
                         *[ptr(t) for t in self.fields()], ptr(self.flux_reg),
                         *[ptr(t) for t in acc])


class Plan:
    """Owns a ppm_plan; the methods mirror the C functions of the same names."""

    def __init__(self, patches: list, nlevels: int = 1, precision: int = PPM_FP64,
                 prm: ppm_params | None = None, tile_config: str | None = None, stream=None):
        self._patches = list(patches)  # keep the tensors alive
        arr = (ppm_patch * len(patches))(*[p.to_c() for p in patches])
        self.params = prm if prm is not None else params()
        self.nlevels = nlevels
        self.precision = precision
        h = _vp()
        cfg = tile_config.encode() if tile_config else None
        _check(lib().ppm_plan_create(C.byref(h), arr, len(patches), nlevels, precision,
                                     C.byref(self.params), cfg, _stream_handle(stream)),
               "ppm_plan_create")
        self._h = h

    def ppm_fill_periodic(self, stream=None):
        _check(lib().ppm_fill_periodic(self._h, _stream_handle(stream)), "ppm_fill_periodic")

    def ppm_fill_boundary(self, patch, kinds, inflow=None, stream=None):
        """Ghost fill of one patch by per-face boundary conditions (PPM_FACE_*,
        faces -x,+x,-y,+y,-z,+z); inflow: [6 faces][rho, vx, vy, vz, etot, eint]."""
        k = (C.c_int32 * 6)(*[int(v) for v in kinds])
        inf = None
        if inflow is not None:
            vals = [float(v) for row in inflow for v in row]
            if len(vals) != 36:
                raise ValueError("inflow must be 6 faces x 6 fields")
            inf = (C.c_double * 36)(*vals)
        _check(lib().ppm_fill_boundary(self._h, int(patch), k, inf, _stream_handle(stream)),
               "ppm_fill_boundary")

    def ppm_set_hierarchy(self, places, stream=None):
        """places: per patch (parent index or -1, refinement factor, (start x, y, z))."""
        arr = (ppm_patch_place * len(places))()
        for i, (parent, refine, start) in enumerate(places):
            arr[i].parent, arr[i].refine = int(parent), int(refine)
            for a in range(3):
                arr[i].start[a] = int(start[a])
        _check(lib().ppm_set_hierarchy(self._h, arr, _stream_handle(stream)), "ppm_set_hierarchy")

    def ppm_fill_ghosts(self, level, stream=None):
        _check(lib().ppm_fill_ghosts(self._h, int(level), _stream_handle(stream)), "ppm_fill_ghosts")

    def ppm_set_expansion(self, a_dev):
        """a_dev: float64 device tensor of 2 * nlevels values (a, adot per
        level), kept alive by the plan; None restores the static equations."""
        self._expand = a_dev
        _check(lib().ppm_set_expansion(self._h, None if a_dev is None else a_dev.data_ptr()),
               "ppm_set_expansion")

    def ppm_expansion(self, dt_dev, stream=None):
        _check(lib().ppm_expansion(self._h, dt_dev.data_ptr(), _stream_handle(stream)),
               "ppm_expansion")

    def ppm_cfl_dt(self, dt_dev, stream=None):
        _check(lib().ppm_cfl_dt(self._h, dt_dev.data_ptr(), _stream_handle(stream)), "ppm_cfl_dt")

    def ppm_step(self, dt_dev, sweep_order=0, stream=None):
        sweep_order = ORDERS.get(sweep_order, sweep_order)
        _check(lib().ppm_step(self._h, dt_dev.data_ptr(), int(sweep_order),
                              _stream_handle(stream)), "ppm_step")

    def ppm_step_cfl(self, dt_dev, sweep_order=0, stream=None):
        sweep_order = ORDERS.get(sweep_order, sweep_order)
        _check(lib().ppm_step_cfl(self._h, dt_dev.data_ptr(), int(sweep_order),
                                  _stream_handle(stream)), "ppm_step_cfl")

    def ppm_sweep(self, dt_dev, axis: int, active_mask: int, stream=None):
        _check(lib().ppm_sweep(self._h, dt_dev.data_ptr(), axis, active_mask,
                               _stream_handle(stream)), "ppm_sweep")

    def ppm_sweep_cfl(self, dt_dev, axis: int, active_mask: int, stream=None):
        _check(lib().ppm_sweep_cfl(self._h, dt_dev.data_ptr(), axis, active_mask,
                                   _stream_handle(stream)), "ppm_sweep_cfl")

    def ppm_cfl_finalize(self, dt_dev, stream=None):
        _check(lib().ppm_cfl_finalize(self._h, dt_dev.data_ptr(), _stream_handle(stream)),
               "ppm_cfl_finalize")

    def ppm_event_counts(self, reset=False, stream=None):
        a, b = C.c_int64(0), C.c_int64(0)
        _check(lib().ppm_event_counts(self._h, C.byref(a), C.byref(b), int(bool(reset)),
                                      _stream_handle(stream)), "ppm_event_counts")
        return a.value, b.value

    def close(self):
        if getattr(self, "_h", None):
            lib().ppm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Amr:
    """Owns a ppm_amr: the W-cycle over a static hierarchy of patches.

    places: per patch (parent index or -1, refinement factor, (start x, y, z)),
    as for Plan.ppm_set_hierarchy; root_kinds / root_inflow: the root's domain
    boundary conditions (None: periodic)."""

    def __init__(self, patches: list, places: list, nlevels: int, precision: int = PPM_FP64,
                 prm: ppm_params | None = None, root_kinds=None, root_inflow=None, stream=None):
        self._patches = list(patches)
        self.nlevels = nlevels
        arr = (ppm_patch * len(patches))(*[p.to_c() for p in patches])
        pl = (ppm_patch_place * len(places))()
        for i, (parent, refine, start) in enumerate(places):
            pl[i].parent, pl[i].refine = int(parent), int(refine)
            for a in range(3):
                pl[i].start[a] = int(start[a])
        self.params = prm if prm is not None else params()
        kinds = None if root_kinds is None else (C.c_int32 * 6)(*[int(k) for k in root_kinds])
        inflow = None
        if root_inflow is not None:
            inflow = (C.c_double * 36)(*[float(v) for row in root_inflow for v in row])
        h = _vp()
        _check(lib().ppm_amr_create(C.byref(h), arr, pl, len(patches), nlevels, precision,
                                    C.byref(self.params), kinds, inflow, _stream_handle(stream)),
               "ppm_amr_create")
        self._h = h

    def ppm_amr_set_expansion(self, a_dev):
        """a_dev: float64 device tensor of 2 * nlevels values, kept alive here."""
        self._expand = a_dev
        _check(lib().ppm_amr_set_expansion(self._h, None if a_dev is None else a_dev.data_ptr()),
               "ppm_amr_set_expansion")

    def ppm_amr_step(self, stream=None):
        _check(lib().ppm_amr_step(self._h, _stream_handle(stream)), "ppm_amr_step")

    def ppm_amr_times(self):
        t = (C.c_double * self.nlevels)()
        n = (C.c_int64 * self.nlevels)()
        _check(lib().ppm_amr_times(self._h, t, n), "ppm_amr_times")
        return list(t), list(n)

    def ppm_amr_step_log(self):
        cnt = C.c_int32(0)
        _check(lib().ppm_amr_step_log(self._h, None, None, 0, C.byref(cnt)), "ppm_amr_step_log")
        lv = (C.c_int32 * max(cnt.value, 1))()
        dt = (C.c_double * max(cnt.value, 1))()
        _check(lib().ppm_amr_step_log(self._h, lv, dt, cnt.value, C.byref(cnt)),
               "ppm_amr_step_log")
        return [(lv[i], dt[i]) for i in range(cnt.value)]

    def ppm_amr_event_counts(self, stream=None):
        a, b = C.c_int64(0), C.c_int64(0)
        _check(lib().ppm_amr_event_counts(self._h, C.byref(a), C.byref(b),
                                          _stream_handle(stream)), "ppm_amr_event_counts")
        return a.value, b.value

    def close(self):
        if getattr(self, "_h", None):
            lib().ppm_amr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A captured step (ppm_graph_create); launch() replays it."""

    def __init__(self, plan: Plan, dt_dev, sweep_order=0, parts=PPM_GRAPH_CFL | PPM_GRAPH_STEP,
                 stream=None):
        sweep_order = ORDERS.get(sweep_order, sweep_order)
        self._plan, self._dt = plan, dt_dev  # keep alive
        h = _vp()
        _check(lib().ppm_graph_create(C.byref(h), plan._h, dt_dev.data_ptr(), int(sweep_order),
                                      int(parts), _stream_handle(stream)), "ppm_graph_create")
        self._h = h

    def ppm_graph_launch(self, stream=None):
        _check(lib().ppm_graph_launch(self._h, _stream_handle(stream)), "ppm_graph_launch")

    def close(self):
        if getattr(self, "_h", None):
            lib().ppm_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
