"""Shared test helpers: move seeded inputs to the device and back, and compare
HIP results with the oracle's."""
from __future__ import annotations

import numpy as np

FIELDS = ("rho", "vx", "vy", "vz", "etot", "eint")


def to_device(d: dict, precision: int, ghost: int = 3, dx=None, level: int = 0,
              with_reg: bool = False):
    """numpy field dict -> ppm.Patch of CUDA tensors (rounded to the storage type)."""
    import torch
    from paper_1307_2265_amd import ppm
    low = torch.float32 if precision == ppm.PPM_MIXED else torch.float64
    t = {}
    for f in FIELDS:
        dt = torch.float64 if f in ("etot", "eint") else low
        t[f] = torch.from_numpy(np.ascontiguousarray(d[f])).to("cuda", dtype=dt).contiguous()
    nz, ny, nx = (s - 2 * ghost for s in d["rho"].shape)
    if dx is None:
        dx = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    reg = None
    if with_reg:
        reg = torch.zeros(ppm.ppm_flux_reg_size(nx, ny, nz), dtype=torch.float64, device="cuda")
    return ppm.Patch(**t, dx=dx[0], dy=dx[1], dz=dx[2], ghost=ghost, level=level, flux_reg=reg)


def to_device_flat(fields: list, precision: int, dxs: list, levels: list,
                   with_reg: bool = False, ghost: int = 3) -> list:
    """Patches as views into one device array per field (patches back to back),
    the layout a batched caller keeps its patches in."""
    import torch
    from paper_1307_2265_amd import ppm
    low = torch.float32 if precision == ppm.PPM_MIXED else torch.float64
    flat = {}
    for f in FIELDS:
        dt = torch.float64 if f in ("etot", "eint") else low
        host = np.concatenate([np.ascontiguousarray(d[f]).ravel() for d in fields])
        flat[f] = torch.from_numpy(host).to("cuda", dtype=dt)
    out, off = [], 0
    for d, dx, lev in zip(fields, dxs, levels):
        shape = d["rho"].shape
        size = int(np.prod(shape))
        views = {f: flat[f][off:off + size].view(shape) for f in FIELDS}
        nz, ny, nx = (s - 2 * ghost for s in shape)
        reg = None
        if with_reg:
            reg = torch.zeros(ppm.ppm_flux_reg_size(nx, ny, nz), dtype=torch.float64,
                              device="cuda")
        out.append(ppm.Patch(**views, dx=dx[0], dy=dx[1], dz=dx[2], ghost=ghost, level=lev,
                             flux_reg=reg))
        off += size
    return out


def from_device(p) -> dict:
    return {f: getattr(p, f).double().cpu().numpy() for f in FIELDS}


def stored_inputs(d: dict, precision: int) -> dict:
    """The values the device actually stores, as float64 (the oracle's input)."""
    from paper_1307_2265_amd import ppm
    out = {}
    for f in FIELDS:
        a = np.ascontiguousarray(d[f], dtype=np.float64)
        if precision == ppm.PPM_MIXED and f not in ("etot", "eint"):
            a = a.astype(np.float32).astype(np.float64)
        out[f] = a
    return out


def oracle_grid(O, d: dict, ghost: int = 3, dx=None, with_reg=False):
    d = {f: np.array(d[f], dtype=np.float64, copy=True) for f in FIELDS}
    nz, ny, nx = (s - 2 * ghost for s in d["rho"].shape)
    if dx is None:
        dx = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    G = O.Grid(**d, dx=dx[0], dy=dx[1], dz=dx[2], ghost=ghost)
    if with_reg:
        G.flux_reg = np.zeros(O.flux_reg_size(nx, ny, nz))
    return G


def rel_err(gpu: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """|g - o| / max(|o|, mean |o|) per cell (relative error with a floor for
    values near zero, e.g. velocities)."""
    scale = np.maximum(np.abs(ref), np.mean(np.abs(ref)))
    scale = np.where(scale > 0, scale, 1.0)
    return np.abs(gpu - ref) / scale


def compare_fields(gpu: dict, ref: dict, tol: float, region=None):
    """Return (worst relative error, cells not bitwise equal) over all fields."""
    worst, differ = 0.0, 0
    for f in FIELDS:
        a, b = gpu[f], ref[f]
        if region is not None:
            a, b = a[region], b[region]
        assert np.all(np.isfinite(a)), f
        e = rel_err(a, b)
        worst = max(worst, float(e.max()))
        differ += int(np.count_nonzero(a != b))
        assert e.max() <= tol, (f, float(e.max()), np.unravel_index(int(e.argmax()), e.shape))
    return worst, differ
