"""Oracle: TEST INFRASTRUCTURE ONLY.

A plain FP64 CPU implementation of the dimensionally split PPM update of the
Enzo method paper (arXiv:1307.2265, Sec. "Hydrodynamics: The PPM method",
"The dual energy formulation", "Riemann Solvers and Fallback", and the hydro
CFL of Sec. "Timestepping"), plus an exact Riemann solver used to pin it.
The arithmetic lives in ``ppm_oracle.cpp`` / ``exact_riemann.cpp``; this module
only builds that library and marshals numpy arrays into it.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this package.  It shares no code with the HIP path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["ppm_oracle.cpp", "exact_riemann.cpp"]

STEEPEN, FLATTEN, DUAL_ENERGY, FALLBACK_HLL = 1, 2, 4, 8
HLLC = 16  # HLLC face fluxes instead of the two-shock solver
DIFFUSION = 32  # CW84's diffusive flux where the flow converges
ALL_FLAGS = STEEPEN | FLATTEN | DUAL_ENERGY | FALLBACK_HLL
ORDERS = {"xyz": 0, "zyx": 1, "xzy": 2, "yxz": 3, "yzx": 4, "zxy": 5}


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with g++ (-O2, no FP contraction, no fast-math)."""
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", _LIB_PATH + ".tmp"]
    cmd += [os.path.join(_HERE, s) for s in _SOURCES]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double), ("eta1", C.c_double),
                ("eta2", C.c_double), ("rho_floor", C.c_double), ("p_floor", C.c_double),
                ("e_floor", C.c_double), ("riemann_rtol", C.c_double),
                ("riemann_max_iter", C.c_int32), ("flags", C.c_uint32),
                ("a", C.c_double), ("adot", C.c_double)]


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("ghost", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)] + \
               [(f, C.POINTER(C.c_double)) for f in
                ("rho", "vx", "vy", "vz", "etot", "eint", "flux_reg", "gx", "gy", "gz")]


class Box(C.Structure):
    """Active cells [lo, hi) of a grid (a finer patch's footprint)."""
    _fields_ = [("lo", C.c_int32 * 3), ("hi", C.c_int32 * 3)]


def box(lo, hi) -> Box:
    return Box((C.c_int32 * 3)(*[int(v) for v in lo]), (C.c_int32 * 3)(*[int(v) for v in hi]))


def box_reg_size(b: Box) -> int:
    return flux_reg_size(*[b.hi[a] - b.lo[a] for a in range(3)])


class Counts(C.Structure):
    _fields_ = [("fallback_faces", C.c_int64), ("floored_cells", C.c_int64)]


def params(gamma=5.0 / 3.0, cfl=0.4, eta1=1e-3, eta2=0.1, rho_floor=1e-20, p_floor=1e-20,
           e_floor=1e-30, riemann_rtol=1e-13, riemann_max_iter=20, flags=ALL_FLAGS,
           a=1.0, adot=0.0) -> Params:
    return Params(gamma, cfl, eta1, eta2, rho_floor, p_floor, e_floor, riemann_rtol,
                  riemann_max_iter, flags, a, adot)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.ppmo_flux_reg_size.restype = C.c_int64
        L.ppmo_flux_reg_size.argtypes = [C.c_int32] * 3
        L.ppmo_step.argtypes = [C.POINTER(_Grid), C.POINTER(Params), C.c_double, C.c_int32,
                                C.POINTER(Counts)]
        L.ppmo_sweep.argtypes = [C.POINTER(_Grid), C.POINTER(Params), C.c_double, C.c_int32,
                                 C.c_int32, C.POINTER(Counts)]
        L.ppmo_pencil.argtypes = [C.POINTER(Params), C.c_int32, C.c_int32, C.c_double,
                                  C.c_double] + \
            [dp] * 8 + [C.POINTER(Counts)]
        L.ppmo_cfl_signal_max.restype = C.c_double
        L.ppmo_cfl_signal_max.argtypes = [C.POINTER(_Grid), C.POINTER(Params)]
        L.ppmo_cfl_dt.restype = C.c_double
        L.ppmo_cfl_dt.argtypes = [C.POINTER(_Grid), C.POINTER(Params)]
        L.ppmo_fill_periodic.argtypes = [C.POINTER(_Grid)]
        L.ppmo_expansion.argtypes = [C.POINTER(_Grid), C.POINTER(Params), C.c_double]
        L.ppmo_fill_boundary.argtypes = [C.POINTER(_Grid), C.POINTER(C.c_int32), dp]
        L.ppmo_second_order_a.argtypes = [dp, C.c_int32, dp]
        L.ppmo_step_capture.argtypes = [C.POINTER(_Grid), C.POINTER(Params), C.c_double,
                                        C.c_int32, C.POINTER(Counts), C.POINTER(Box), C.c_int32,
                                        dp]
        L.ppmo_flux_correct.argtypes = [C.POINTER(_Grid), C.POINTER(Params), C.POINTER(Box),
                                        C.c_int32, dp, dp, C.c_int32]
        L.ppmo_project.argtypes = [C.POINTER(_Grid), C.POINTER(Box), C.POINTER(_Grid),
                                   C.c_int32]
        L.ppmo_fill_from_parent.argtypes = [C.POINTER(_Grid), C.POINTER(C.c_int32),
                                            C.POINTER(_Grid), C.POINTER(C.c_int32), C.c_int32]
        L.ppmo_copy_from_sibling.argtypes = [C.POINTER(_Grid), C.POINTER(C.c_int32),
                                             C.POINTER(_Grid), C.POINTER(C.c_int32)]
        L.ppmo_two_shock.argtypes = [C.POINTER(Params), dp, dp, dp]
        L.ppmo_hll_flux.argtypes = [C.POINTER(Params), dp, dp, dp]
        L.ppmo_hllc_flux.argtypes = [C.POINTER(Params), dp, dp, dp]
        L.ppmo_exact_riemann.argtypes = [C.c_double, dp, dp, C.c_int32, dp, dp, dp, dp, dp]
        L.ppmo_count_ops.argtypes = [C.POINTER(_Grid), C.POINTER(Params), C.c_double, C.c_int32,
                                     C.POINTER(C.c_int64)]
        L.ppmo_num_threads.restype = C.c_int
        L.ppmo_set_num_threads.argtypes = [C.c_int32]
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return C.POINTER(C.c_double)()
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


FIELDS = ("rho", "vx", "vy", "vz", "etot", "eint")


@dataclass
class Grid:
    """Host-side grid: six float64 arrays of shape (nz+6, ny+6, nx+6)."""
    rho: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    etot: np.ndarray
    eint: np.ndarray
    dx: float
    dy: float
    dz: float
    ghost: int = 3
    flux_reg: np.ndarray | None = None
    accel: tuple | None = None  # (gx, gy, gz) at the cell centres, same shape as the fields

    @property
    def active_shape(self):
        g = self.ghost
        nz, ny, nx = self.rho.shape
        return nx - 2 * g, ny - 2 * g, nz - 2 * g

    def fields(self):
        return [getattr(self, f) for f in FIELDS]

    def copy(self) -> "Grid":
        return Grid(*[f.copy() for f in self.fields()], self.dx, self.dy, self.dz, self.ghost,
                    None if self.flux_reg is None else self.flux_reg.copy(),
                    None if self.accel is None else tuple(a.copy() for a in self.accel))

    def _c(self) -> _Grid:
        nx, ny, nz = self.active_shape
        for f in self.fields() + list(self.accel or ()):
            assert f.dtype == np.float64 and f.flags.c_contiguous and f.shape == self.rho.shape
        acc = [_ptr(a) for a in self.accel] if self.accel is not None else [None] * 3
        return _Grid(nx, ny, nz, self.ghost, self.dx, self.dy, self.dz,
                     *[_ptr(f) for f in self.fields()], _ptr(self.flux_reg), *acc)


def expansion(grid: Grid, prm: Params, dt: float) -> None:
    """The split expansion terms of the comoving equations over dt (active cells)."""
    g = grid._c()
    if lib().ppmo_expansion(C.byref(g), C.byref(prm), float(dt)) != 0:
        raise ValueError("ppmo_expansion: invalid argument")


def flux_reg_size(nx, ny, nz) -> int:
    return int(lib().ppmo_flux_reg_size(nx, ny, nz))


def step(grid: Grid, prm: Params, dt: float, order: int | str = 0) -> Counts:
    order = ORDERS.get(order, order)
    c = Counts(0, 0)
    g = grid._c()
    rc = lib().ppmo_step(C.byref(g), C.byref(prm), dt, int(order), C.byref(c))
    if rc != 0:
        raise ValueError("ppmo_step: invalid argument")
    return c


def sweep(grid: Grid, prm: Params, dt: float, axis: int, active_mask: int) -> Counts:
    c = Counts(0, 0)
    g = grid._c()
    rc = lib().ppmo_sweep(C.byref(g), C.byref(prm), dt, axis, active_mask, C.byref(c))
    if rc != 0:
        raise ValueError("ppmo_sweep: invalid argument")
    return c


def pencil(prm: Params, dt: float, dx: float, rho, u, v1, v2, etot, eint, want_reg=False,
           ghost: int = 3):
    """Sweep one 1-D pencil in place; returns (counts, reg_lo, reg_hi)."""
    n = len(rho)
    lo = np.zeros(6) if want_reg else None
    hi = np.zeros(6) if want_reg else None
    c = Counts(0, 0)
    rc = lib().ppmo_pencil(C.byref(prm), n, ghost, dt, dx,
                           *[_ptr(a) for a in (rho, u, v1, v2, etot, eint)],
                           _ptr(lo), _ptr(hi), C.byref(c))
    if rc != 0:
        raise ValueError("ppmo_pencil: invalid argument")
    return c, lo, hi


def cfl_signal_max(grid: Grid, prm: Params) -> float:
    g = grid._c()
    return float(lib().ppmo_cfl_signal_max(C.byref(g), C.byref(prm)))


def cfl_dt(grid: Grid, prm: Params) -> float:
    g = grid._c()
    return float(lib().ppmo_cfl_dt(C.byref(g), C.byref(prm)))


FACE_PERIODIC, FACE_REFLECTING, FACE_OUTFLOW, FACE_INFLOW = 0, 1, 2, 3


def fill_boundary(grid: Grid, kinds, inflow=None) -> None:
    """Ghost fill by per-face boundary conditions (faces -x,+x,-y,+y,-z,+z);
    inflow: [6 faces][rho, vx, vy, vz, etot, eint] for INFLOW faces."""
    k = (C.c_int32 * 6)(*[int(v) for v in kinds])
    inf = None
    if inflow is not None:
        inf = np.ascontiguousarray(inflow, dtype=np.float64).reshape(36)
    g = grid._c()
    if lib().ppmo_fill_boundary(C.byref(g), k, None if inf is None else _ptr(inf)) != 0:
        raise ValueError("ppmo_fill_boundary: invalid argument")


def second_order_a(nb, r: int) -> np.ndarray:
    """SecondOrderA values [k][j][i] of the centre of a 3x3x3 neighbourhood [dz][dy][dx]."""
    a = np.ascontiguousarray(nb, dtype=np.float64).reshape(27)
    out = np.zeros(r ** 3)
    lib().ppmo_second_order_a(_ptr(a), int(r), _ptr(out))
    return out.reshape(r, r, r)


def step_capture(grid: Grid, prm: Params, dt: float, order, boxes: list) -> tuple:
    """ppmo_step that also returns the fluxes dt*F through the faces of each
    box (list of Box), one register-shaped block per box, concatenated."""
    order = ORDERS.get(order, order)
    c = Counts(0, 0)
    arr = (Box * max(len(boxes), 1))(*boxes)
    out = np.zeros(max(sum(box_reg_size(b) for b in boxes), 1))
    g = grid._c()
    if lib().ppmo_step_capture(C.byref(g), C.byref(prm), dt, int(order), C.byref(c), arr,
                               len(boxes), _ptr(out)) != 0:
        raise ValueError("ppmo_step_capture: invalid argument")
    return c, out[:sum(box_reg_size(b) for b in boxes)]


def flux_correct(coarse: Grid, prm: Params, boxes: list, caps: np.ndarray,
                 fine_sums: np.ndarray, r: int) -> None:
    arr = (Box * max(len(boxes), 1))(*boxes)
    caps = np.ascontiguousarray(caps, dtype=np.float64)
    fine_sums = np.ascontiguousarray(fine_sums, dtype=np.float64)
    g = coarse._c()
    if lib().ppmo_flux_correct(C.byref(g), C.byref(prm), arr, len(boxes), _ptr(caps),
                               _ptr(fine_sums), int(r)) != 0:
        raise ValueError("ppmo_flux_correct: invalid argument")


def project(coarse: Grid, b: Box, fine: Grid, r: int) -> None:
    gc, gf = coarse._c(), fine._c()
    if lib().ppmo_project(C.byref(gc), C.byref(b), C.byref(gf), int(r)) != 0:
        raise ValueError("ppmo_project: invalid argument")


def fill_from_parent(fine: Grid, fine_start, parent: Grid, parent_start, r: int) -> None:
    fs = (C.c_int32 * 3)(*[int(v) for v in fine_start])
    ps = (C.c_int32 * 3)(*[int(v) for v in parent_start])
    gf, gp = fine._c(), parent._c()
    if lib().ppmo_fill_from_parent(C.byref(gf), fs, C.byref(gp), ps, int(r)) != 0:
        raise ValueError("ppmo_fill_from_parent: invalid argument")


def copy_from_sibling(dst: Grid, dst_start, src: Grid, src_start) -> None:
    ds = (C.c_int32 * 3)(*[int(v) for v in dst_start])
    ss = (C.c_int32 * 3)(*[int(v) for v in src_start])
    gd, gs = dst._c(), src._c()
    if lib().ppmo_copy_from_sibling(C.byref(gd), ds, C.byref(gs), ss) != 0:
        raise ValueError("ppmo_copy_from_sibling: invalid argument")


def fill_periodic(grid: Grid) -> None:
    g = grid._c()
    if lib().ppmo_fill_periodic(C.byref(g)) != 0:
        raise ValueError("ppmo_fill_periodic: invalid argument")


def two_shock(prm: Params, left, right) -> dict:
    l = np.ascontiguousarray(left, dtype=np.float64)
    r = np.ascontiguousarray(right, dtype=np.float64)
    out = np.zeros(7)
    lib().ppmo_two_shock(C.byref(prm), _ptr(l), _ptr(r), _ptr(out))
    return dict(p_star=out[0], u_star=out[1], rho=out[2], u=out[3], p=out[4],
                iters=int(out[5]), left=bool(out[6]))


def hll_flux(prm: Params, left6, right6) -> np.ndarray:
    l = np.ascontiguousarray(left6, dtype=np.float64)
    r = np.ascontiguousarray(right6, dtype=np.float64)
    out = np.zeros(7)
    lib().ppmo_hll_flux(C.byref(prm), _ptr(l), _ptr(r), _ptr(out))
    return out


def hllc_flux(prm: Params, left6, right6) -> np.ndarray:
    """HLLC flux on traced states (rho, u, v1, v2, p): F_rho, F_u, F_v1, F_v2,
    F_E, F_e and the face velocity (S* inside the fan)."""
    l = np.ascontiguousarray(left6, dtype=np.float64)
    r = np.ascontiguousarray(right6, dtype=np.float64)
    out = np.zeros(7)
    lib().ppmo_hllc_flux(C.byref(prm), _ptr(l), _ptr(r), _ptr(out))
    return out


def exact_riemann(gamma: float, left, right, xi) -> tuple:
    """Exact Riemann solution sampled at x/t = xi; returns (rho, u, p, star)."""
    l = np.ascontiguousarray(left, dtype=np.float64)
    r = np.ascontiguousarray(right, dtype=np.float64)
    xi = np.ascontiguousarray(np.atleast_1d(xi), dtype=np.float64)
    rho, u, p, star = (np.zeros(len(xi)), np.zeros(len(xi)), np.zeros(len(xi)), np.zeros(4))
    lib().ppmo_exact_riemann(gamma, _ptr(l), _ptr(r), len(xi), _ptr(xi), _ptr(rho), _ptr(u),
                             _ptr(p), _ptr(star))
    return rho, u, p, dict(p_star=star[0], u_star=star[1], rho_star_l=star[2],
                           rho_star_r=star[3])


def count_ops(grid: Grid, prm: Params, dt: float, order: int | str = 0) -> dict:
    """Algorithmic operation counts of one step (advances the grid)."""
    order = ORDERS.get(order, order)
    ops = (C.c_int64 * 6)()
    g = grid._c()
    if lib().ppmo_count_ops(C.byref(g), C.byref(prm), dt, int(order), ops) != 0:
        raise ValueError("ppmo_count_ops: invalid argument")
    return dict(add=ops[0], mul=ops[1], div=ops[2], sqrt=ops[3], cmp=ops[4], cell_sweeps=ops[5])


def num_threads() -> int:
    return int(lib().ppmo_num_threads())


def set_num_threads(n: int) -> None:
    """Host threads of later calls (results do not depend on it)."""
    lib().ppmo_set_num_threads(int(n))
