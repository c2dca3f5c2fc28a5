"""Oracle of the AMR level step on a static patch hierarchy (test
infrastructure only, like the rest of `oracle/`).

The W-cycle of Sec. "Adaptive Mesh Refinement" (EvolveLevel): beginning with
the root, every level takes one step over all its patches, then its children
advance as many steps as they need to reach its time, after which the level
is corrected with the children's boundary fluxes (Sec. "Flux correction")
and the children's values are projected onto the cells they cover
(Sec. "Projection").  Ghost zones are set at the start and after every step
of a level: the root's by its domain boundary conditions, a finer patch's by
SecondOrderA interpolation from its parent's state at the patch's time --
linear in time between the parent's states before and after its step --
followed by copies from siblings.  Each level's timestep is the hydro CFL
step of its patches (Sec. "Timestepping"), cut so that the level lands on its
parent's time exactly.

Readings (the paper shows the control flow, not these details):
  * the time interpolation blends the stored fields, (1 - w) q_old + w q_new
    with w = (t - t_old) / (t_new - t_old) of the parent (so w = 0 and w = 1
    reproduce the two states exactly), before the spatial interpolation;
  * the fine fluxes are summed over the substeps (each patch's register holds
    dt F of its last step) and area-averaged over the r^2 fine faces of a
    coarse face; all six register quantities (rho, rho v, rho E and the
    advective part of rho e) are corrected;
  * a child's footprint lies at least one cell inside its parent's active
    region, so every corrected cell belongs to the parent;
  * the sweep order alternates xyz / zyx with each step of a level;
  * a step whose CFL timestep reaches the parent's time takes exactly the
    remaining interval and lands on the parent's time;
  * in comoving coordinates each level uses its own a, adot (its params), and
    a level step applies the split expansion terms to its active cells after
    its sweeps, over the same dt (before the ghost zones are set again).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import (FIELDS, Grid, box, box_reg_size, cfl_signal_max, copy_from_sibling,
               fill_boundary, fill_from_parent, fill_periodic, flux_correct, flux_reg_size,
               project, step, step_capture)
from . import expansion as expansion_step


@dataclass
class Node:
    grid: Grid
    level: int
    parent: int = -1           # index of the parent node (-1: the root)
    start: tuple = (0, 0, 0)   # global index of the first active cell, in its level
    r: int = 2                 # refinement factor from the parent's cells


@dataclass
class Hierarchy:
    nodes: list
    params: list               # one oracle Params per level (a, adot of that level)
    root_kinds: list | None = None   # domain boundary kinds of the root (None: periodic)
    root_inflow: object = None       # [face][rho, vx, vy, vz, etot, eint] of inflow faces
    correct: bool = True       # flux correction on (off only for negative controls)
    expansion: bool = False    # apply the comoving expansion terms after each level step
    t: list = field(default_factory=list)
    t_old: list = field(default_factory=list)
    nsteps: list = field(default_factory=list)
    dts: list = field(default_factory=list)   # (level, dt) of every step taken

    def __post_init__(self):
        L = 1 + max(n.level for n in self.nodes)
        self.L = L
        self.t = [0.0] * L
        self.t_old = [0.0] * L
        self.nsteps = [0] * L
        roots = [i for i, n in enumerate(self.nodes) if n.level == 0]
        if len(roots) != 1:
            raise ValueError("one root patch on level 0")
        self.children = {i: [] for i in range(len(self.nodes))}
        for i, n in enumerate(self.nodes):
            if n.level > 0:
                p = self.nodes[n.parent]
                if p.level != n.level - 1:
                    raise ValueError("a parent is one level coarser")
                if n.grid.flux_reg is None:
                    raise ValueError("patches below the root need flux registers")
                self.children[n.parent].append(i)
        self.boxes = {i: [self.footprint(c) for c in ch] for i, ch in self.children.items()}
        # the siblings each patch copies ghost cells from, in patch order
        self.neighbours = {i: [j for j in self.level(n.level) if j != i and self._may_touch(i, j)]
                           for i, n in enumerate(self.nodes)}
        self.acc = {i: np.zeros(flux_reg_size(*n.grid.active_shape))
                    for i, n in enumerate(self.nodes) if n.level > 0}
        self.old = {}

    def level(self, l):
        return [i for i, n in enumerate(self.nodes) if n.level == l]

    def footprint(self, c):
        """Box of the parent's active cells that child c covers."""
        n = self.nodes[c]
        p = self.nodes[n.parent]
        dims = n.grid.active_shape  # (nx, ny, nz)
        lo, hi = [], []
        for a in range(3):
            if n.start[a] % n.r or dims[a] % n.r:
                raise ValueError("a child starts and ends on parent cell boundaries")
            lo.append(n.start[a] // n.r - p.start[a])
            hi.append(lo[a] + dims[a] // n.r)
        return box(lo, hi)

    # -- boundary values -----------------------------------------------------
    def _parent_at(self, p, t, cache):
        """The parent's stored fields at time t, linear in time between its
        states before and after its last step (cache: blends already made
        for this fill, by parent)."""
        P = self.nodes[p]
        l = P.level
        if self.t[l] == self.t_old[l] or p not in self.old:
            return P.grid
        if p not in cache:
            w = (t - self.t_old[l]) / (self.t[l] - self.t_old[l])
            old = self.old[p]
            blend = {f: (1.0 - w) * getattr(old, f) + w * getattr(P.grid, f) for f in FIELDS}
            g = P.grid
            cache[p] = Grid(**blend, dx=g.dx, dy=g.dy, dz=g.dz, ghost=g.ghost)
        return cache[p]

    def fill(self, l):
        ids = self.level(l)
        if l == 0:
            root = self.nodes[ids[0]].grid
            if self.root_kinds is None:
                fill_periodic(root)
            else:
                fill_boundary(root, self.root_kinds, self.root_inflow)
            return
        cache = {}
        for i in ids:
            n = self.nodes[i]
            src = self._parent_at(n.parent, self.t[l], cache)
            fill_from_parent(n.grid, n.start, src, self.nodes[n.parent].start, n.r)
        for i in ids:
            for j in self.neighbours[i]:
                copy_from_sibling(self.nodes[i].grid, self.nodes[i].start,
                                  self.nodes[j].grid, self.nodes[j].start)

    def _may_touch(self, i, j):
        """Whether patch j's active box meets patch i's ghosted box (else the
        sibling copy from j to i copies nothing)."""
        a, b = self.nodes[i], self.nodes[j]
        da, db = a.grid.active_shape, b.grid.active_shape
        g = a.grid.ghost
        return all(a.start[k] - g < b.start[k] + db[k] and b.start[k] < a.start[k] + da[k] + g
                   for k in range(3))

    # -- the W-cycle ---------------------------------------------------------
    def cfl_dt(self, l):
        prm = self.params[l]
        s = max(cfl_signal_max(self.nodes[i].grid, prm) for i in self.level(l))
        return (prm.cfl * prm.a) / s

    def evolve(self, l=0, t_end=None):
        """EvolveLevel: one step of the root (t_end None), else steps of level l
        until it reaches t_end."""
        ids = self.level(l)
        prm = self.params[l]
        self.fill(l)
        while t_end is None or self.t[l] < t_end:
            dt = self.cfl_dt(l)
            t_new = self.t[l] + dt
            if t_end is not None and dt >= t_end - self.t[l]:
                dt = t_end - self.t[l]
                t_new = t_end
            self.dts.append((l, dt))
            order = self.nsteps[l] % 2
            caps = {}
            for i in ids:
                g = self.nodes[i].grid
                if self.children[i]:
                    self.old[i] = g.copy()
                    _, caps[i] = step_capture(g, prm, dt, order, self.boxes[i])
                else:
                    step(g, prm, dt, order)
                if l > 0:
                    self.acc[i] = self.acc[i] + g.flux_reg
            if self.expansion:
                for i in ids:
                    expansion_step(self.nodes[i].grid, prm, dt)
            self.t_old[l] = self.t[l]
            self.t[l] = t_new
            self.nsteps[l] += 1
            self.fill(l)
            if l + 1 < self.L:
                self.evolve(l + 1, self.t[l])
                for i in ids:
                    ch = self.children[i]
                    if not ch:
                        continue
                    r = self.nodes[ch[0]].r
                    if self.correct:
                        sums = np.concatenate([self.acc[c] for c in ch])
                        flux_correct(self.nodes[i].grid, prm, self.boxes[i], caps[i], sums, r)
                    for c in ch:
                        self.acc[c][:] = 0.0
                    for c, b in zip(ch, self.boxes[i]):
                        project(self.nodes[i].grid, b, self.nodes[c].grid, self.nodes[c].r)
            if t_end is None:
                break

    # -- diagnostics ---------------------------------------------------------
    def composite_totals(self):
        """Mass, momentum and total energy of the composite solution: every
        patch's active cells not covered by a child, times the cell volume."""
        tot = np.zeros(5)
        for i, n in enumerate(self.nodes):
            g = n.grid
            gh = g.ghost
            act = (slice(gh, -gh),) * 3
            mask = np.ones(g.rho[act].shape, bool)
            for b in self.boxes[i]:
                mask[b.lo[2]:b.hi[2], b.lo[1]:b.hi[1], b.lo[0]:b.hi[0]] = False
            rho = g.rho[act][mask]
            vol = g.dx * g.dy * g.dz
            tot += vol * np.array([rho.sum(), (rho * g.vx[act][mask]).sum(),
                                   (rho * g.vy[act][mask]).sum(),
                                   (rho * g.vz[act][mask]).sum(),
                                   (rho * g.etot[act][mask]).sum()])
        return tot


__all__ = ["Node", "Hierarchy", "box_reg_size"]
