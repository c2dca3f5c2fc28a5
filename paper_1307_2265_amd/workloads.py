"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds none of the method's arithmetic: it draws random primitive
fields and converts them to the stored variables (density, velocity, specific
total energy E = p/((gamma-1) rho) + |v|^2/2 and specific internal energy
e = p/((gamma-1) rho)), which is the definition of the initial state.  Ghost
zones are left at zero for periodic grids (each path fills its own), or drawn
like the active cells for patches whose ghosts are seeded.

Recipe (numpy PCG64, one generator per grid; whole arrays are drawn in C
order (z, y, x) in the order rho, vx, vy, vz, p):
  * density: mean-one lognormal, rho = exp(sigma Z - sigma^2/2);
  * velocity: independent Gaussians per component with standard deviation
    vel_sigma * c_ref, c_ref = sqrt(gamma <p>/<rho>) = sqrt(gamma);
  * pressure: 1 + amp U(-1, 1) ("uniform") or a mean-one lognormal.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

GAMMA = 5.0 / 3.0
GHOST = 3


@dataclass(frozen=True)
class FieldRecipe:
    rho_sigma: float          # sigma of ln(rho)
    vel_sigma: float          # per-component std of v in units of c_ref
    p_kind: str               # "uniform" or "lognormal"
    p_param: float            # amplitude (uniform) or sigma of ln(p)


# config 0/1: gentle white noise; config 2/3: strongly shocked (rms Mach 5).
GENTLE = FieldRecipe(0.5, 0.5, "uniform", 0.1)
SHOCKED = FieldRecipe(2.0, 5.0 / np.sqrt(3.0), "lognormal", 1.0)


def _draw(rng: np.random.Generator, shape, recipe: FieldRecipe, gamma: float):
    c_ref = np.sqrt(gamma)
    s = recipe.rho_sigma
    rho = np.exp(s * rng.standard_normal(shape) - 0.5 * s * s)
    v = [recipe.vel_sigma * c_ref * rng.standard_normal(shape) for _ in range(3)]
    if recipe.p_kind == "uniform":
        p = 1.0 + recipe.p_param * rng.uniform(-1.0, 1.0, shape)
    else:
        sp = recipe.p_param
        p = np.exp(sp * rng.standard_normal(shape) - 0.5 * sp * sp)
    return rho, v, p


def stored_from_primitive(rho, vx, vy, vz, p, gamma: float):
    """(rho, v, p) -> stored fields (rho, vx, vy, vz, E, e)."""
    e = p / ((gamma - 1.0) * rho)
    etot = e + 0.5 * (vx * vx + vy * vy + vz * vz)
    return rho, vx, vy, vz, etot, e


def random_grid(nx: int, ny: int, nz: int, seed: int, recipe: FieldRecipe = GENTLE,
                gamma: float = GAMMA, seeded_ghosts: bool = False,
                ghost: int = GHOST) -> dict:
    """Return dict of six float64 arrays of shape (nz+2g, ny+2g, nx+2g).

    With seeded_ghosts=False only the active cells are drawn and the ghosts
    are zero (to be filled periodically); otherwise the whole box is drawn.
    """
    g = ghost
    full = (nz + 2 * g, ny + 2 * g, nx + 2 * g)
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = full if seeded_ghosts else (nz, ny, nx)
    rho, (vx, vy, vz), p = _draw(rng, shape, recipe, gamma)
    stored = stored_from_primitive(rho, vx, vy, vz, p, gamma)
    out = {}
    for name, a in zip(("rho", "vx", "vy", "vz", "etot", "eint"), stored):
        if seeded_ghosts:
            out[name] = np.ascontiguousarray(a, dtype=np.float64)
        else:
            b = np.zeros(full)
            b[g:g + nz, g:g + ny, g:g + nx] = a
            out[name] = b
    return out


def vacuum_pockets(d: dict, seed: int, frac: float = 0.05, speed: float = 100.0,
                   rho_vac: float = 1e-20, p_vac: float = 1e-20, gamma: float = GAMMA,
                   ghost: int = GHOST) -> dict:
    """Turn a seeded fraction of the active cells of d (in place) into
    near-vacuum cells: density rho_vac, pressure p_vac (the default floors) and
    normally distributed velocities of standard deviation speed.  Such cells
    next to dense moving gas drive the reconstructed edge density or pressure
    to zero."""
    g = ghost
    act = (slice(g, -g),) * 3
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = d["rho"][act].shape
    vac = rng.random(shape) < frac
    prim = {k: np.array(d[k][act]) for k in ("rho", "vx", "vy", "vz", "eint")}
    p = (gamma - 1.0) * prim["rho"] * prim["eint"]
    prim["rho"][vac] = rho_vac
    p[vac] = p_vac
    for k in ("vx", "vy", "vz"):
        prim[k][vac] = rng.normal(0.0, speed, int(vac.sum()))
    st = stored_from_primitive(prim["rho"], prim["vx"], prim["vy"], prim["vz"], p, gamma)
    for k, a in zip(("rho", "vx", "vy", "vz", "etot", "eint"), st):
        d[k][act] = a
    return d


def uniform_grid(nx, ny, nz, rho, v, p, gamma=GAMMA, ghost=GHOST) -> dict:
    g = ghost
    full = (nz + 2 * g, ny + 2 * g, nx + 2 * g)
    st = stored_from_primitive(np.float64(rho), np.float64(v[0]), np.float64(v[1]),
                               np.float64(v[2]), np.float64(p), gamma)
    return {n: np.full(full, a, dtype=np.float64)
            for n, a in zip(("rho", "vx", "vy", "vz", "etot", "eint"), st)}


# ---------------------------------------------------------------------------
# Batched AMR patches (uneven sizes and levels, seeded ghosts).

PATCH_DIMS = (8, 12, 16, 24, 32)


@dataclass
class PatchSpec:
    nx: int
    ny: int
    nz: int
    level: int
    dx: float
    seed: int


def patch_specs(npatch: int, seed: int, max_level: int = 6, dims=PATCH_DIMS) -> list:
    """Per-axis dims i.i.d. from `dims`, level uniform in 0..max_level, dx = 2^-level."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.choice(np.asarray(dims), size=(npatch, 3))
    lev = rng.integers(0, max_level + 1, size=npatch)
    sub = rng.integers(0, 2**62, size=npatch)
    return [PatchSpec(int(a), int(b), int(c), int(l), 2.0 ** -int(l), int(s))
            for (a, b, c), l, s in zip(d, lev, sub)]


def patch_fields(spec: PatchSpec, recipe: FieldRecipe = SHOCKED, gamma: float = GAMMA) -> dict:
    return random_grid(spec.nx, spec.ny, spec.nz, spec.seed, recipe, gamma, seeded_ghosts=True)


def acceleration_field(shape, seed: int, amp: float = 1.0, modes: int = 4, device=None,
                       dtype=None) -> tuple:
    """Three arrays of `shape` (z, y, x), a smooth seeded acceleration field:
    per component, a sum of `modes` plane waves over the array's cell indices
    with wave numbers drawn from 1..3 per axis (in units of 2 pi over the
    array extent), random phases and standard normal amplitudes, scaled by
    amp / sqrt(modes).  numpy float64 arrays, or, with `device`, torch tensors
    of `dtype` (default float64) evaluated there from the same draws."""
    rng = np.random.Generator(np.random.PCG64(seed))
    draws = [[(rng.integers(1, 4, size=3), rng.uniform(0.0, 2.0 * np.pi), rng.standard_normal())
              for _ in range(modes)] for _ in range(3)]
    if device is None:
        axes = [np.arange(n, dtype=np.float64) / n for n in shape]
        sin, zeros, cast = np.sin, (lambda: np.zeros(shape)), np.ascontiguousarray
    else:
        import torch
        axes = [torch.arange(n, dtype=torch.float64, device=device) / n for n in shape]
        sin = torch.sin
        zeros = lambda: torch.zeros(shape, dtype=torch.float64, device=device)
        cast = lambda t: t.to(dtype or torch.float64).contiguous()
    z, y, x = axes[0][:, None, None], axes[1][None, :, None], axes[2][None, None, :]
    out = []
    for comp in draws:
        g = zeros()
        for k, ph, amp_k in comp:
            g += amp_k * sin(2.0 * np.pi * (int(k[0]) * z + int(k[1]) * y + int(k[2]) * x) + ph)
        out.append(cast(g * (amp / np.sqrt(modes))))
    return tuple(out)


# ---------------------------------------------------------------------------
# Named workloads.

WORKLOADS = {
    "gentle32": dict(n=32, recipe=GENTLE, seed=1000, steps=1),
    "gentle256": dict(n=256, recipe=GENTLE, seed=1001, steps=10),
    "shocked512": dict(n=512, recipe=SHOCKED, seed=1002, steps=20),
}


# ---------------------------------------------------------------------------
# Cosmology-shaped hierarchy: a periodic root grid holding a log-normal
# Gaussian random field density and cold bulk flows, plus nested patches on
# levels 1-8 whose fields (ghosts included) are injected piecewise constant
# from the root at random positions.  The root is generated on the GPU with
# torch (white noise filtered in Fourier space), so these inputs exist only
# where a GPU does; the CPU oracle receives copies of the generated arrays.

# Grids per level in the paper's AMR scaling run (Sec. "AMR scaling"),
# levels 1-6, extended to levels 7 and 8 by the ratio 0.7 per level.
HIER_LEVEL_WEIGHTS = (61868.0, 91182.0, 59932.0, 40700.0, 28346.0, 19771.0,
                      19771.0 * 0.7, 19771.0 * 0.49)
HIER_DIMS = tuple(range(16, 49, 2))   # per-axis active dims of a patch
HIER_RHO_SIGMA = 1.5                  # sigma of ln(rho)
HIER_KE_OVER_TE_MAX = 1e6             # largest kinetic / thermal energy ratio


@dataclass
class HierPatch:
    nx: int
    ny: int
    nz: int
    level: int
    dx: float
    origin: tuple   # root cell (x, y, z) of the patch's first active cell


def hierarchy_specs(npatch: int, n_root: int, seed: int) -> list:
    """Patch dims i.i.d. from HIER_DIMS, levels 1-8 drawn with the weights
    above, dx = 2^-level / n_root, origin uniform over the root's cells."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = np.asarray(HIER_LEVEL_WEIGHTS)
    lev = rng.choice(np.arange(1, 9), size=npatch, p=w / w.sum())
    d = rng.choice(np.asarray(HIER_DIMS), size=(npatch, 3))
    org = rng.integers(0, n_root, size=(npatch, 3))
    return [HierPatch(int(a), int(b), int(c), int(l), 2.0 ** -int(l) / n_root,
                      (int(o[0]), int(o[1]), int(o[2])))
            for (a, b, c), l, o in zip(d, lev, org)]


def _grf(n: int, gen, device):
    """Unit-variance Gaussian random field on an n^3 periodic grid with power
    spectrum P(k) ~ k^-2 (white noise times 1/|k| in Fourier space, k = 0
    removed)."""
    import torch
    w = torch.randn((n, n, n), generator=gen, dtype=torch.float64, device=device)
    F = torch.fft.rfftn(w)
    del w
    k = torch.fft.fftfreq(n, d=1.0 / n, dtype=torch.float64, device=device)
    kr = torch.fft.rfftfreq(n, d=1.0 / n, dtype=torch.float64, device=device)
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + kr[None, None, :] ** 2
    k2[0, 0, 0] = 1.0
    F *= k2.rsqrt_()
    F[0, 0, 0] = 0.0
    del k2
    d = torch.fft.irfftn(F, s=(n, n, n))
    del F
    d -= d.mean()
    d /= d.std()
    return d


def hierarchy_root(n: int, seed: int, gamma: float = GAMMA, device="cuda",
                   ghost: int = GHOST) -> dict:
    """Root fields as float64 device tensors of shape (n+2g)^3 with zero ghosts:
    rho = exp(1.5 delta - 1.125) (mean one), three velocity components that
    are independent unit-variance fields of the same spectrum, and a cold
    adiabatic gas e = e_c rho^(gamma-1) with e_c such that the largest
    kinetic / thermal energy ratio over the grid is 1e6."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    s = HIER_RHO_SIGMA
    full = (n + 2 * ghost,) * 3
    inner = (slice(ghost, ghost + n),) * 3
    out = {}
    rho = torch.exp(s * _grf(n, gen, device) - 0.5 * s * s)
    ke = torch.zeros((n, n, n), dtype=torch.float64, device=device)
    for name in ("vx", "vy", "vz"):
        v = _grf(n, gen, device)
        ke += 0.5 * v * v
        out[name] = torch.zeros(full, dtype=torch.float64, device=device)
        out[name][inner] = v
        del v
    rg = rho ** (gamma - 1.0)
    ec = float((ke / rg).max()) / HIER_KE_OVER_TE_MAX
    e = ec * rg
    del rg
    for name, a in (("rho", rho), ("eint", e), ("etot", e + ke)):
        out[name] = torch.zeros(full, dtype=torch.float64, device=device)
        out[name][inner] = a
    return out


def inject_patch(root: dict, spec: HierPatch, n_root: int, ghost: int = GHOST) -> dict:
    """A patch's fields (ghosts included) injected piecewise constant from the
    root's active cells: patch cell i along an axis lies in root cell
    origin + floor((i - g) / 2^level), wrapped periodically."""
    import torch
    dev = root["rho"].device
    r = 2 ** spec.level

    def idx(n, o):
        i = torch.arange(n + 2 * ghost, device=dev) - ghost
        return (o + torch.div(i, r, rounding_mode="floor")) % n_root + ghost

    ix, iy, iz = idx(spec.nx, spec.origin[0]), idx(spec.ny, spec.origin[1]), idx(spec.nz, spec.origin[2])
    sel = (iz[:, None, None], iy[None, :, None], ix[None, None, :])
    return {k: v[sel] for k, v in root.items()}


# ---------------------------------------------------------------------------
# A nested hierarchy for the patch ghost fill: a root grid, and on each finer
# level (refinement 2) blocks of dims[l]^3 cells laid on a lattice inside every
# patch of the level above, abutting each other (so siblings cover each
# other's ghost cells) and kept `margin` parent cells away from the parent's
# active edge.  Only the geometry; fields come from random_grid.

@dataclass
class NestedPatch:
    level: int
    parent: int          # index in the list, -1 for the root
    start: tuple         # global index of the first active cell in its level
    dims: tuple


def nested_hierarchy(n_root: int, dims: tuple, per_axis: tuple, margin: int = 2) -> list:
    """dims[l], per_axis[l]: block size and lattice of level l + 1."""
    out = [NestedPatch(0, -1, (0, 0, 0), (n_root,) * 3)]
    frontier = [0]
    for lev in range(1, len(dims) + 1):
        dim, per = dims[lev - 1], per_axis[lev - 1]
        nxt = []
        for pi in frontier:
            par = out[pi]
            span = per * dim // 2                            # parent cells the block lattice covers
            room = par.dims[0] - 2 * margin - span
            if room < 0:
                continue
            o = [par.start[a] + margin + room // 2 for a in range(3)]
            for k in range(per):
                for j in range(per):
                    for i in range(per):
                        start = (2 * o[0] + i * dim, 2 * o[1] + j * dim, 2 * o[2] + k * dim)
                        out.append(NestedPatch(lev, pi, start, (dim, dim, dim)))
                        nxt.append(len(out) - 1)
        frontier = nxt
    return out
