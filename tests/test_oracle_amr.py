"""Pins of the oracle's AMR level step on a static hierarchy (CPU only).

The W-cycle (Sec. "Adaptive Mesh Refinement"), flux correction (Sec. "Flux
correction") and projection (Sec. "Projection") are pinned by what the paper
fixes independently of their code: the composite solution of a periodic
hierarchy conserves mass, momentum and total energy to round-off over a root
step with subcycled levels (and does not without the correction -- the
negative control shows the pin bites); a hierarchy of one level is plain
stepping, bit for bit; the face fluxes a step records for a box equal the
flux registers of a grid that is exactly that box; projection conserves the
mass of what it averages; the parent state a child's ghosts see is linear in
time between the parent's states; and a smooth contact advected through a
refined region is more accurate on the fine patch than on the coarse grid
alone, with the refined run's coarse cells no worse than the unrefined run's.
The paper's shock pool and wave pool (Sec. "Shock pool", "Wave pool") pin
the hierarchy on its own test problems: the shock crosses the refined region
at the exact speed, and a short linear sound wave enters and leaves it
without a reflection, at the speed of sound.
"""
import numpy as np
import pytest

from oracle import amr
from paper_1307_2265_amd import workloads as W

GH = 4


def _grid(O, d, dx, ghost=GH, reg=False):
    nz, ny, nx = (s - 2 * ghost for s in d["rho"].shape)
    G = O.Grid(**{k: np.ascontiguousarray(v) for k, v in d.items()}, dx=dx[0], dy=dx[1],
               dz=dx[2], ghost=ghost)
    if reg:
        G.flux_reg = np.zeros(O.flux_reg_size(nx, ny, nz))
    return G


def _nested(O, seed, recipe=W.GENTLE, siblings=False):
    """Periodic 16^3 root, a level-1 child and a level-2 grandchild (r = 2),
    each at least one parent cell inside its parent; siblings adds a second
    level-1 child that does not touch the first."""
    spec = [(0, -1, (0, 0, 0), (16, 16, 16)),
            (1, 0, (8, 8, 8), (12, 12, 12)),
            (2, 1, (20, 20, 20), (8, 8, 8))]
    if siblings:
        spec.append((1, 0, (2, 22, 4), (8, 6, 10)))
    nodes = []
    for i, (lev, par, start, dims) in enumerate(spec):
        d = W.random_grid(*dims, seed + i, recipe, ghost=GH)
        h = 1.0 / 16 * 0.5 ** lev
        nodes.append(amr.Node(_grid(O, d, (h, h, h), reg=lev > 0), lev, par, start, 2))
    return nodes


def test_composite_conservation_over_a_root_step(O):
    H = amr.Hierarchy(_nested(O, 500, siblings=True), [O.params()] * 3)
    H.fill(0)
    for l in (1, 2):
        H.fill(l)
    t0 = H.composite_totals()
    for _ in range(2):
        H.evolve()
    t1 = H.composite_totals()
    # several substeps of each finer level per root step
    assert sum(1 for l, _ in H.dts if l == 2) > sum(1 for l, _ in H.dts if l == 0)
    scale = np.array([t0[0], t0[0], t0[0], t0[0], t0[4]])
    assert np.all(np.abs(t1 - t0) <= 1e-13 * scale), (t1 - t0) / scale


def test_without_flux_correction_conservation_fails(O):
    H = amr.Hierarchy(_nested(O, 500, siblings=True), [O.params()] * 3, correct=False)
    for l in (0, 1, 2):
        H.fill(l)
    t0 = H.composite_totals()
    H.evolve()
    t1 = H.composite_totals()
    assert abs(t1[0] - t0[0]) > 1e-9 * t0[0]


def test_one_level_is_plain_stepping(O):
    d = W.random_grid(12, 10, 8, 510, W.SHOCKED, ghost=GH)
    A = _grid(O, {k: v.copy() for k, v in d.items()}, (1 / 12, 1 / 10, 1 / 8))
    B = _grid(O, {k: v.copy() for k, v in d.items()}, (1 / 12, 1 / 10, 1 / 8))
    prm = O.params()
    H = amr.Hierarchy([amr.Node(A, 0)], [prm])
    for s in range(3):
        H.evolve()
        O.fill_periodic(B)
        dt = O.cfl_dt(B, prm)
        O.step(B, prm, dt, s % 2)
        assert H.dts[-1] == (0, dt)
    O.fill_periodic(B)
    for f in O.FIELDS:
        assert np.array_equal(getattr(A, f), getattr(B, f)), f


def test_captured_fluxes_of_a_whole_grid_box_are_its_registers(O):
    d = W.random_grid(10, 8, 6, 520, W.SHOCKED, ghost=GH)
    A = _grid(O, {k: v.copy() for k, v in d.items()}, (0.1, 0.125, 1 / 6), reg=True)
    B = _grid(O, {k: v.copy() for k, v in d.items()}, (0.1, 0.125, 1 / 6), reg=True)
    O.fill_periodic(A)
    O.fill_periodic(B)
    prm = O.params()
    dt = O.cfl_dt(A, prm)
    sub = O.box((2, 1, 3), (7, 6, 5))
    _, cap = O.step_capture(A, prm, dt, 1, [O.box((0, 0, 0), (10, 8, 6)), sub])
    O.step(B, prm, dt, 1)
    n0 = O.flux_reg_size(10, 8, 6)
    assert np.array_equal(cap[:n0], B.flux_reg)
    for f in O.FIELDS:
        assert np.array_equal(getattr(A, f), getattr(B, f))
    # an interior box: its -x face fluxes are the ones that cross x = 2 - 1/2
    assert np.abs(cap[n0:]).max() > 0


def test_projection_conserves_the_mass_it_averages(O):
    d = W.random_grid(8, 8, 8, 530, W.SHOCKED, ghost=GH)
    C = _grid(O, d, (0.125,) * 3)
    f = W.random_grid(6, 4, 8, 531, W.SHOCKED, ghost=GH)
    F = _grid(O, f, (0.0625,) * 3)
    b = O.box((2, 3, 1), (5, 5, 5))
    fact = (slice(GH, -GH),) * 3
    fine = [F.rho[fact].sum() * F.dx ** 3, (F.rho * F.vx)[fact].sum() * F.dx ** 3,
            (F.rho * F.etot)[fact].sum() * F.dx ** 3]
    O.project(C, b, F, 2)
    cs = (slice(GH + 1, GH + 5), slice(GH + 3, GH + 5), slice(GH + 2, GH + 5))
    coarse = [C.rho[cs].sum() * C.dx ** 3, (C.rho * C.vx)[cs].sum() * C.dx ** 3,
              (C.rho * C.etot)[cs].sum() * C.dx ** 3]
    for a, c in zip(fine, coarse):
        assert c == pytest.approx(a, rel=1e-13, abs=1e-15)
    # cells outside the box are untouched
    assert np.array_equal(C.rho[GH, GH, GH], d["rho"][GH, GH, GH])


def test_child_ghosts_see_the_parent_linearly_in_time(O):
    # a uniform parent at 1.0 before its step and 2.0 after it: a child at a
    # quarter of the step sees 1.25 in every ghost cell
    nodes = _nested(O, 540)[:2]
    for n in nodes:
        for f in O.FIELDS:
            getattr(n.grid, f)[...] = 1.0
    H = amr.Hierarchy(nodes, [O.params()] * 2)
    H.old[0] = nodes[0].grid.copy()
    nodes[0].grid.rho[...] = 2.0
    H.t_old[0], H.t[0] = 0.0, 1.0
    H.t[1] = 0.25
    H.fill(1)
    g = nodes[1].grid
    assert np.all(g.rho[:GH] == 1.25) and np.all(g.rho[GH:-GH, GH:-GH, GH:-GH] == 1.0)
    # momentum and energy densities are interpolated; v = (rho v) / rho = 1
    assert np.allclose(g.vx[:GH], 1.0, rtol=1e-15)


def _contact(nx, ny, nz, x0, dx, ghost=GH, amp=0.2):
    """rho = 1 + amp sin(2 pi x) at the cell centres (x0: global x of the first
    active cell's left face), v = (1, 0, 0), p = 1."""
    x = x0 + (np.arange(nx + 2 * ghost) - ghost + 0.5) * dx
    shape = (nz + 2 * ghost, ny + 2 * ghost, nx + 2 * ghost)
    rho = np.broadcast_to(1.0 + amp * np.sin(2 * np.pi * x), shape).copy()
    one, zero = np.ones(shape), np.zeros(shape)
    st = W.stored_from_primitive(rho, one, zero, zero.copy(), one.copy(), 5.0 / 3.0)
    return dict(zip(("rho", "vx", "vy", "vz", "etot", "eint"), st))


def test_smooth_contact_is_more_accurate_on_the_refined_patch(O):
    n = 32
    h = 1.0 / n
    prm = O.params()
    root = _grid(O, _contact(n, 8, 8, 0.0, h), (h, h, h))
    ref = _grid(O, _contact(n, 8, 8, 0.0, h), (h, h, h))
    # child: coarse x 8..24, y 1..7, z 1..7 (r = 2)
    child = _grid(O, _contact(32, 12, 12, 8 * h, h / 2), (h / 2,) * 3, reg=True)
    H = amr.Hierarchy([amr.Node(root, 0), amr.Node(child, 1, 0, (16, 2, 2), 2)], [prm, prm])
    T = 0.25
    while H.t[0] < T - 1e-12:
        H.evolve()
    t = H.t[0]
    # the unrefined run to the same time, with the same root steps
    s = 0
    for l, dt in H.dts:
        if l == 0:
            O.fill_periodic(ref)
            O.step(ref, prm, dt, s % 2)
            s += 1
    exact = lambda x: 1.0 + 0.2 * np.sin(2 * np.pi * (x - t))
    xc = (np.arange(n) + 0.5) * h
    xf = 8 * h + (np.arange(32) + 0.5) * h / 2
    a = (slice(GH, -GH),) * 3
    err_f = np.abs(child.rho[a][3, 3] - exact(xf)).mean()
    err_c = np.abs(ref.rho[a][3, 3, 8:24] - exact(xc[8:24])).mean()
    out = np.r_[0:7, 25:32]
    err_out_h = np.abs(root.rho[a][3, 3, out] - exact(xc[out])).mean()
    err_out_c = np.abs(ref.rho[a][3, 3, out] - exact(xc[out])).mean()
    assert err_f < 0.5 * err_c, (err_f, err_c)
    assert err_out_h < 1.5 * err_out_c, (err_out_h, err_out_c)


def _shock_pool(O, refined: bool):
    """Sec. "Shock pool": gas at rest (rho = p = 1, gamma = 1.4) on x in [0, 1]
    (100 root cells; 4 cells across, periodic in y and z), a Mach-2 shock
    driven in from the left boundary (inflow of the post-shock state, outflow
    on the right), a static refined region from x = 0.25 to 0.75 (r = 2; one
    root cell of margin across)."""
    g, gam, M = 3, 1.4, 2.0
    rho2 = (gam + 1) * M * M / ((gam - 1) * M * M + 2)
    p2 = (2 * gam * M * M - (gam - 1)) / (gam + 1)
    S = M * np.sqrt(gam)
    u2 = S * (1 - 1 / rho2)
    e2 = p2 / ((gam - 1) * rho2)
    inflow = np.zeros((6, 6))
    inflow[0] = [rho2, u2, 0.0, 0.0, e2 + 0.5 * u2 * u2, e2]
    def uniform(nx, ny, nz):
        shape = (nz + 2 * g, ny + 2 * g, nx + 2 * g)
        one, zero = np.ones(shape), np.zeros(shape)
        st = W.stored_from_primitive(one, zero, zero.copy(), zero.copy(), one.copy(), gam)
        return dict(zip(O.FIELDS, [np.ascontiguousarray(a) for a in st]))
    prm = O.params(gamma=gam)
    h = 0.01
    nodes = [amr.Node(_grid(O, uniform(100, 4, 4), (h, h, h), ghost=g), 0)]
    if refined:
        nodes.append(amr.Node(_grid(O, uniform(100, 4, 4), (h / 2,) * 3, ghost=g, reg=True), 1, 0,
                              (50, 2, 2), 2))
    kinds = [3, 2, 0, 0, 0, 0]
    H = amr.Hierarchy(nodes, [prm] * len(nodes), root_kinds=kinds, root_inflow=inflow)
    return H, (rho2, S)


def test_shock_pool_keeps_the_shock_on_both_levels(O):
    # the shock enters and leaves the refined region at the exact speed, on
    # the fine and the coarse cells, with the unrefined run's plateau
    H, (rho2, S) = _shock_pool(O, True)
    U, _ = _shock_pool(O, False)
    g = 3
    def front(grid, x0, dx):
        r = grid.rho[g + 1, g + 1, g:-g]       # a row inside the refined region in y, z
        i = int(np.argmax(r < 0.5 * (1 + rho2)))
        return x0 + i * dx
    for t_check in (0.2, 0.35):
        while H.t[0] < t_check - 1e-12:
            H.evolve()
        while U.t[0] < t_check - 1e-12:
            U.evolve()
        xs = S * H.t[0]
        root, fine = H.nodes[0].grid, H.nodes[1].grid
        assert abs(front(root, 0.0, 0.01) - xs) <= 0.02, (t_check, front(root, 0.0, 0.01), xs)
        assert abs(front(U.nodes[0].grid, 0.0, 0.01) - S * U.t[0]) <= 0.02
        if t_check == 0.2:                     # inside the refined region
            assert abs(front(fine, 0.25, 0.005) - xs) <= 0.01, (front(fine, 0.25, 0.005), xs)
        # post-shock plateau behind the front, on the root
        plat = root.rho[g + 1, g + 1, g + 5:g + int(100 * xs) - 5]
        assert np.all(np.abs(plat - rho2) < 0.05 * rho2), plat
    # the region the shock has crossed and left agrees with the unrefined run
    a = H.nodes[0].grid.rho[g + 1, g + 1, g + 5:g + 70]
    b = U.nodes[0].grid.rho[g + 1, g + 1, g + 5:g + 70]
    assert np.abs(a - b).max() < 0.05 * rho2


def _wave_pool(O, refined: bool):
    """Sec. "Wave pool": gas at rest (rho = p = 1, gamma = 1.4) on x in [0, 1]
    (100 root cells; 4 cells across, periodic in y and z), a static refined
    region from x = 0.25 to 0.75 (r = 2; one root cell of margin across),
    outflow at both x faces.  The paper drives the wave in through the left
    boundary; here the same right-moving linear sound wave (amplitude
    A = 0.01, wavelength 0.1, i.e. 10 root cells) starts as a train of two
    wavelengths on 0.02 <= x < 0.22: rho = 1 + A s, u = c0 A s,
    p = 1 + gamma A s with s = sin(2 pi (x - 0.02) / 0.1), c0 = sqrt(gamma)."""
    g, gam, A = 3, 1.4, 0.01
    c0 = np.sqrt(gam)
    def wave(nx, dx, x_lo):
        shape = (4 + 2 * g, 4 + 2 * g, nx + 2 * g)
        x = x_lo + (np.arange(nx + 2 * g) - g + 0.5) * dx
        s = np.where((x >= 0.02) & (x < 0.22), np.sin(2 * np.pi * (x - 0.02) / 0.1), 0.0)
        z = np.zeros(shape)
        st = W.stored_from_primitive(np.broadcast_to(1 + A * s, shape).copy(),
                                     np.broadcast_to(c0 * A * s, shape).copy(), z, z.copy(),
                                     np.broadcast_to(1 + gam * A * s, shape).copy(), gam)
        return dict(zip(O.FIELDS, [np.ascontiguousarray(a) for a in st]))
    h = 0.01
    nodes = [amr.Node(_grid(O, wave(100, h, 0.0), (h, h, h), ghost=g), 0)]
    if refined:
        nodes.append(amr.Node(_grid(O, wave(100, h / 2, 0.25), (h / 2,) * 3, ghost=g, reg=True),
                              1, 0, (50, 2, 2), 2))
    H = amr.Hierarchy(nodes, [O.params(gamma=gam)] * len(nodes), root_kinds=[2, 2, 0, 0, 0, 0])
    return H, (A, c0)


def test_wave_pool_passes_the_refined_region_cleanly(O):
    # checked on the root as the paper plots it, before the wave enters
    # (t = 0.2), once it is wholly inside (0.3) and wholly past the exit (0.64):
    # the left-moving characteristic field the refined region adds to the
    # unrefined run's stays below 1 % of the wave (no reflection), the wave is
    # no more damped than without refinement, and it travels at c0
    H, (A, c0) = _wave_pool(O, True)
    U, _ = _wave_pool(O, False)
    g = 3
    xs = (np.arange(100) + 0.5) * 0.01
    def invariants(grid):
        r = grid.rho[g + 1, g + 1, g:-g]
        u = grid.vx[g + 1, g + 1, g:-g]
        p = 0.4 * r * grid.eint[g + 1, g + 1, g:-g]
        return u + (p - 1) / c0, u - (p - 1) / c0      # right- and left-moving, linearised
    amp = 2 * c0 * A
    for t_check in (0.2, 0.3, 0.64):
        while H.t[0] < t_check - 1e-12:
            H.evolve()
        while U.t[0] < t_check - 1e-12:
            U.evolve()
        jp, jm = invariants(H.nodes[0].grid)
        jpu, jmu = invariants(U.nodes[0].grid)
        behind = ((xs < 0.25) | (xs >= 0.75)) & (xs < 0.02 + c0 * H.t[0] - 0.03)
        if behind.any():
            assert np.abs(jm - jmu)[behind].max() < 0.01 * amp, t_check
        assert np.abs(jp).max() >= np.abs(jpu).max(), t_check
        centroid = (xs * np.abs(jp)).sum() / np.abs(jp).sum()
        assert abs(centroid - (0.12 + c0 * H.t[0])) < 0.015, (t_check, centroid)
