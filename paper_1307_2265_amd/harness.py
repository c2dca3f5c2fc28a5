"""Device-side workload setup and timing shared by bench.py and the autotuner.

Builds the seeded workloads of workloads.py on the GPU (a single periodic
grid, or a batch of uneven patches stored as views into one flat buffer per
field), runs steps through the C ABI and times them with HIP events on the
launch stream.  A step is fill (periodic grids) -> the three sweeps, the last
of which also yields the next step's CFL timestep (ppm_step_cfl, directly or
as a captured HIP graph); the first step's timestep comes from a plain CFL
reduction (ppm_cfl_dt), issued whenever the state was reset.
"""
from __future__ import annotations

import numpy as np

from . import ppm
from . import workloads as W

FIELDS = ("rho", "vx", "vy", "vz", "etot", "eint")
ORDERS = ((0, 1, 2), (2, 1, 0))  # xyz on even steps, zyx on odd ones


def _torch():
    import torch
    return torch


def lanes_mask_of(tiles: str | None) -> int:
    if tiles and "lanes=" in tiles:
        return int(tiles.split("lanes=")[1].split()[0])
    return 1


class Run:
    """Patches, plan and per-level dt array of one workload on the device."""

    def __init__(self, host_fields: list, specs: list, prec: int, nlevels: int, periodic: bool,
                 tiles: str | None = None, with_reg: bool = False, ghost: int = W.GHOST,
                 flags: int | None = None, sources: dict | None = None):
        """sources (optional): dict(seed=, amp=, a=, adot=): every patch gets a
        seeded acceleration field (W.acceleration_field, in rho's type) and
        every level the expansion factor a and rate adot; a step is then the
        expansion terms followed by the sweeps with the gravity sources, both
        over the step's dt."""
        torch = _torch()
        low = torch.float32 if prec == ppm.PPM_MIXED else torch.float64
        self.prec, self.periodic, self.tiles, self.nlevels = prec, periodic, tiles, nlevels
        self.params = ppm.params() if flags is None else ppm.params(flags=flags)
        sizes = [f["rho"].size for f in host_fields]
        offs = np.concatenate([[0], np.cumsum(sizes)])
        self.flat = {}
        for name in FIELDS:
            dt = torch.float64 if name in ("etot", "eint") else low
            host = np.concatenate([f[name].ravel() for f in host_fields])
            self.flat[name] = torch.from_numpy(host).to("cuda", dtype=dt)
        self.init = {k: v.clone() for k, v in self.flat.items()}
        self.reg = None
        if with_reg:
            rs = [ppm.ppm_flux_reg_size(*s[:3]) for s in specs]
            self.reg = torch.zeros(int(sum(rs)), dtype=torch.float64, device="cuda")
            roffs = np.concatenate([[0], np.cumsum(rs)])
        self.patches = []
        for i, (f, sp) in enumerate(zip(host_fields, specs)):
            shape = f["rho"].shape
            views = {k: v[offs[i]:offs[i + 1]].view(shape) for k, v in self.flat.items()}
            reg = None if self.reg is None else self.reg[roffs[i]:roffs[i + 1]]
            nx, ny, nz, level, dx = sp
            acc = None
            if sources is not None:
                acc = W.acceleration_field(shape, sources["seed"] + i, sources["amp"],
                                           device="cuda", dtype=low)
            self.patches.append(ppm.Patch(**views, dx=dx, dy=dx, dz=dx, ghost=ghost,
                                          level=level, flux_reg=reg, accel=acc))
        self.cells = int(sum(s[0] * s[1] * s[2] for s in specs))
        self.expand = None
        if sources is not None:
            self.expand = torch.tensor([sources["a"], sources["adot"]] * nlevels,
                                       dtype=torch.float64, device="cuda")
        self.plan = self._new_plan(tiles)
        self.dt = torch.zeros(nlevels, dtype=torch.float64, device="cuda")
        self.graphs = None
        self.dt_valid = False

    def _new_plan(self, tiles):
        plan = ppm.Plan(self.patches, self.nlevels, self.prec, self.params, tile_config=tiles)
        if self.expand is not None:
            plan.ppm_set_expansion(self.expand)
        return plan

    # -- construction helpers -------------------------------------------------
    @classmethod
    def single(cls, d: dict, n: int, prec: int, tiles=None, flags=None, sources=None):
        return cls([d], [(n, n, n, 0, 1.0 / n)], prec, 1, True, tiles, flags=flags,
                   sources=sources)

    @classmethod
    def batch(cls, specs: list, fields: list, prec: int, tiles=None, nlevels=7):
        sp = [(s.nx, s.ny, s.nz, s.level, s.dx) for s in specs]
        return cls(fields, sp, prec, nlevels, False, tiles, with_reg=True)

    def replan(self, tiles: str | None):
        """Replace the plan by one with other launch shapes (same patches)."""
        if self.graphs:
            for g in self.graphs:
                g.close()
            self.graphs = None
        self.plan.close()
        self.tiles = tiles
        self.plan = self._new_plan(tiles)

    # -- stepping -------------------------------------------------------------
    def reset(self):
        for k, v in self.flat.items():
            v.copy_(self.init[k])
        self.dt_valid = False

    def ensure_dt(self):
        """The current state's CFL timestep in self.dt (a reduction pass),
        unless the last step already left it there."""
        if not self.dt_valid:
            if self.periodic:
                self.plan.ppm_fill_periodic()
            self.plan.ppm_cfl_dt(self.dt)
            self.dt_valid = True

    def step(self, s: int):
        self.ensure_dt()
        if self.expand is not None:  # split expansion terms first, over the same dt
            self.plan.ppm_expansion(self.dt)
        if self.periodic:
            self.plan.ppm_fill_periodic()
        self.plan.ppm_step_cfl(self.dt, s % 2)

    def make_graphs(self):
        parts = ppm.PPM_GRAPH_STEP_CFL
        if self.periodic:
            parts |= ppm.PPM_GRAPH_FILL
        self.graphs = [ppm.Graph(self.plan, self.dt, o, parts) for o in (0, 1)]

    def timed(self, steps: int, graphs: bool = False, per_sweep: bool = False):
        """Time `steps` steps from the current state (its timestep, if not
        known, is reduced before the timed region).

        graphs: replay the captured step graphs.  per_sweep: issue the sweeps
        as ppm_sweep, ppm_sweep, ppm_sweep_cfl + ppm_cfl_finalize bracketed by
        HIP events (the same kernels and extents ppm_step_cfl launches when it
        is not persistent) and return the mean duration per kernel kind
        ("march", "lanes", and "+cfl" for the last sweep's variant, and
        "expansion" for the expansion pass of a run with sources).
        Returns (seconds, {kind: s})."""
        torch = _torch()
        E = lambda: torch.cuda.Event(enable_timing=True)
        if graphs and self.graphs is None:
            self.make_graphs()
        lm = lanes_mask_of(self.tiles)
        ev = []
        self.ensure_dt()
        torch.cuda.synchronize()
        t0, t1 = E(), E()
        t0.record()
        for s in range(steps):
            if graphs:
                if self.expand is not None:
                    self.plan.ppm_expansion(self.dt)
                self.graphs[s % 2].ppm_graph_launch()
                continue
            if not per_sweep:
                self.step(s)
                continue
            if self.expand is not None:
                a, b = E(), E()
                a.record()
                self.plan.ppm_expansion(self.dt)
                b.record()
                ev.append(("expansion", a, b))
            if self.periodic:
                self.plan.ppm_fill_periodic()
            mask = 0
            for k, axis in enumerate(ORDERS[s % 2]):
                a, b = E(), E()
                a.record()
                if k < 2:
                    self.plan.ppm_sweep(self.dt, axis, mask)
                else:
                    self.plan.ppm_sweep_cfl(self.dt, axis, mask)
                b.record()
                kind = "lanes" if (lm >> axis) & 1 else "march"
                ev.append((kind if k < 2 else kind + "+cfl", a, b))
                mask |= 1 << axis
            self.plan.ppm_cfl_finalize(self.dt)
        t1.record()
        torch.cuda.synchronize()
        per = {}
        for kind, a, b in ev:
            per.setdefault(kind, []).append(a.elapsed_time(b) / 1e3)
        return t0.elapsed_time(t1) / 1e3, {k: sum(v) / len(v) for k, v in per.items()}

    def close(self):
        if self.graphs:
            for g in self.graphs:
                g.close()
        self.plan.close()


def active_mask(run: Run):
    """Boolean mask of the active cells in the flat field buffers of a run."""
    torch = _torch()
    m = torch.zeros(run.flat["rho"].numel(), dtype=torch.bool, device="cuda")
    off = 0
    for p in run.patches:
        g = p.ghost
        v = m[off:off + p.rho.numel()].view(p.rho.shape)
        v[g:-g, g:-g, g:-g] = True
        off += p.rho.numel()
    return m


def l1_per_field(a: Run, b: Run) -> dict:
    """sum |a - b| / sum |b| over the active cells of every patch, per field."""
    m = active_mask(b)
    out = {}
    for f in FIELDS:
        x = a.flat[f][m].double()
        y = b.flat[f][m].double()
        out[f] = float((x - y).abs().sum() / y.abs().sum())
    return out


def single_grid_input(n: int, workload: str = "shocked512") -> dict:
    """The seeded single-grid input of a named workload (its recipe and seed
    at n^3 cells), with rho and v rounded to float32 so that both precisions
    start from the same stored values."""
    cfg = W.WORKLOADS[workload]
    d = W.random_grid(n, n, n, cfg["seed"], cfg["recipe"])
    for f in ("rho", "vx", "vy", "vz"):
        d[f] = d[f].astype(np.float32).astype(np.float64)
    return d


def batch_input(npatch: int, seed: int = 1003):
    """Uneven patches (dims from {8,12,16,24,32}, levels 0..6) with seeded ghosts."""
    specs = W.patch_specs(npatch, seed)
    fields = []
    for sp in specs:
        f = W.patch_fields(sp)
        for k in ("rho", "vx", "vy", "vz"):
            f[k] = f[k].astype(np.float32).astype(np.float64)
        fields.append(f)
    return specs, fields


def active(a, ghost: int = W.GHOST):
    """The active block of a ghosted (z, y, x) array."""
    g = ghost
    return a[g:-g, g:-g, g:-g]


def swept_cells(dims: tuple, order: tuple, ghost: int = W.GHOST) -> tuple:
    """(cells written, pencils) of each sweep of one step of a patch with
    active dims (nx, ny, nz) in sweep order `order`: the k-th sweep updates
    the cells active along the axes swept so far and along its own axis and
    every index along the axes still to come."""
    out = []
    done = set()
    for axis in order:
        w = 1
        for t in range(3):
            if t == axis:
                continue
            w *= dims[t] if t in done else dims[t] + 2 * ghost
        out.append((w * dims[axis], w))
        done.add(axis)
    return out


def step_bytes(dims_list, read_b: float, write_b: float, ghost: int = W.GHOST) -> float:
    """Algorithmic HBM bytes of one step over patches of the given active dims
    (the mean of the xyz and zyx orders): every sweep reads each pencil's
    n + 2g cells and writes its n active ones, and the last sweep's
    timestep needs no extra pass."""
    tot = 0.0
    for dims in dims_list:
        for order in ORDERS:
            for (cells, pencils) in swept_cells(dims, order, ghost):
                tot += 0.5 * (cells * (read_b + write_b) + pencils * 2 * ghost * read_b)
    return tot


class Hierarchy:
    """The cosmology-shaped hierarchy on the device: an n_root^3 periodic root
    grid (log-normal Gaussian random field density, cold bulk flows) and
    `npatch` patches of 16^3-48^3 on levels 1-8 with ghosts injected from the
    root, stored as views into one flat buffer per field, flux registers on.
    FP64 or mixed storage."""

    NLEV = 9

    def __init__(self, prec: int, n_root: int = 1024, npatch: int = 20000, seed: int = 1004,
                 ghost: int = W.GHOST, log=None):
        torch = _torch()
        say = log or (lambda m: None)
        G = ghost
        low = torch.float32 if prec == ppm.PPM_MIXED else torch.float64
        self.prec, self.n_root, self.ghost = prec, n_root, ghost
        say(f"generating the {n_root}^3 root")
        root64 = W.hierarchy_root(n_root, seed, ghost=ghost)
        self.specs = W.hierarchy_specs(npatch, n_root, seed)
        sizes = [(s.nz + 2 * G) * (s.ny + 2 * G) * (s.nx + 2 * G) for s in self.specs]
        self.offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        say(f"injecting {npatch} patches ({self.offs[-1] / 1e9:.2f} G cells)")
        self.flat = {f: torch.empty(int(self.offs[-1]), device="cuda",
                                    dtype=torch.float64 if f in ("etot", "eint") else low)
                     for f in FIELDS}
        for i, s in enumerate(self.specs):
            pf = W.inject_patch(root64, s, n_root, ghost)
            for f in FIELDS:
                self.flat[f][self.offs[i]:self.offs[i + 1]].copy_(pf[f].reshape(-1))
            if (i + 1) % 5000 == 0:
                say(f"  {i + 1} patches")
        rsz = [ppm.ppm_flux_reg_size(s.nx, s.ny, s.nz) for s in self.specs]
        self.roffs = np.concatenate([[0], np.cumsum(rsz)]).astype(np.int64)
        self.reg = torch.zeros(int(self.roffs[-1]), dtype=torch.float64, device="cuda")
        self.root = {f: root64[f] if f in ("etot", "eint") else root64[f].to(low)
                     for f in FIELDS}
        del root64
        torch.cuda.empty_cache()
        h = 1.0 / n_root
        self.patches = [ppm.Patch(**self.root, dx=h, dy=h, dz=h, ghost=G, level=0,
                                  bc=ppm.PPM_BC_PERIODIC)]
        for i, s in enumerate(self.specs):
            shape = (s.nz + 2 * G, s.ny + 2 * G, s.nx + 2 * G)
            views = {f: self.flat[f][self.offs[i]:self.offs[i + 1]].view(shape) for f in FIELDS}
            self.patches.append(ppm.Patch(**views, dx=s.dx, dy=s.dx, dz=s.dx, ghost=G,
                                          level=s.level,
                                          flux_reg=self.reg[self.roffs[i]:self.roffs[i + 1]],
                                          bc=ppm.PPM_BC_SUPPLIED))
        self.dims = [(n_root,) * 3] + [(s.nx, s.ny, s.nz) for s in self.specs]
        self.cells = int(sum(a * b * c for a, b, c in self.dims))
