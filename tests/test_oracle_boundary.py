"""Pins of the oracle's domain boundary conditions (CPU only).

The paper's four external boundary conditions (Sec. "Boundary conditions"):
reflecting (mirror image, normal velocity reversed), outflow (copy of the edge
cell), inflow (fixed values) and periodic.  Pins: periodic faces reproduce the
periodic fill; a box with reflecting walls evolves exactly as one half of the
periodic box twice its size that holds the data and its mirror image; a Sod
tube between outflow faces matches the exact solution; a uniform flow entering
through an inflow face and leaving through an outflow face stays uniform.
"""
import numpy as np
import pytest

from paper_1307_2265_amd import workloads as W
from tests.test_oracle_sweeps import _grid

P_, R_, O_, I_ = 0, 1, 2, 3  # periodic, reflecting, outflow, inflow


def _copy(d):
    return {k: v.copy() for k, v in d.items()}


@pytest.mark.parametrize("ghost", [3, 4])
def test_periodic_faces_equal_the_periodic_fill(O, ghost):
    d = W.random_grid(9, 7, 5, 11, W.SHOCKED, ghost=ghost)
    A, B = _grid(O, _copy(d), ghost=ghost), _grid(O, _copy(d), ghost=ghost)
    O.fill_periodic(A)
    O.fill_boundary(B, [P_] * 6)
    for f in O.FIELDS:
        assert np.array_equal(getattr(A, f), getattr(B, f))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_reflecting_walls_evolve_as_half_of_the_mirrored_periodic_box(O, axis):
    # Reflecting walls at both ends of `axis` are the mirror planes of a
    # periodic box twice as long that holds the data and its mirror image
    # (normal velocity negated); both see the same cells, so several steps
    # agree bit for bit (four ghost layers, so that no stencil of the doubled
    # box reaches farther than the walled box's ghosts).
    gh = 4
    prm = O.params()
    dims = [10, 8, 6]
    d = W.random_grid(*dims, 41 + axis, W.SHOCKED, ghost=gh)
    nax = 2 - axis                      # numpy axis of the lab axis
    vel = ("vx", "vy", "vz")[axis]
    act = [slice(gh, -gh)] * 3
    # doubled box: active cells [data, mirror(data)] along the axis
    big = {}
    for f in O.FIELDS:
        a = d[f][tuple(act)]
        m = -np.flip(a, nax) if f == vel else np.flip(a, nax)
        full = np.concatenate([a, m], axis=nax)
        big[f] = np.pad(full, gh, mode="constant")
    dd = dims.copy()
    dd[axis] *= 2
    H = O.Grid(**big, dx=1.0 / dd[0], dy=1.0 / dd[1], dz=1.0 / dd[2], ghost=gh)
    G = O.Grid(**_copy(d), dx=1.0 / dd[0], dy=1.0 / dd[1], dz=1.0 / dd[2], ghost=gh)
    kinds = [P_] * 6
    kinds[2 * axis] = kinds[2 * axis + 1] = R_
    for s in range(3):
        O.fill_periodic(H)
        O.fill_boundary(G, kinds)
        dt_h, dt_g = O.cfl_dt(H, prm), O.cfl_dt(G, prm)
        assert dt_h == dt_g
        O.step(H, prm, dt_h, s % 2)
        O.step(G, prm, dt_g, s % 2)
    half = [slice(gh, -gh)] * 3
    half[nax] = slice(gh, gh + dims[axis])
    for f in O.FIELDS:
        assert np.array_equal(getattr(G, f)[tuple(act)], getattr(H, f)[tuple(half)]), f


def test_reflecting_ghosts_mirror_the_edge_cells(O):
    gh = 3
    d = W.random_grid(5, 4, 6, 12, W.GENTLE, ghost=gh)
    G = _grid(O, _copy(d))
    O.fill_boundary(G, [R_, R_, O_, O_, P_, P_])
    # x: ghost i mirrors active 2*gh-1-i on the low side, with vx negated
    for i in range(gh):
        src = 2 * gh - 1 - i
        assert np.array_equal(G.rho[gh:-gh, gh:-gh, i], G.rho[gh:-gh, gh:-gh, src])
        assert np.array_equal(G.vx[gh:-gh, gh:-gh, i], -G.vx[gh:-gh, gh:-gh, src])
        assert np.array_equal(G.vy[gh:-gh, gh:-gh, i], G.vy[gh:-gh, gh:-gh, src])
    # y outflow over the whole x extent (x ghosts included): copies of the edge row
    for j in range(gh):
        assert np.array_equal(G.etot[gh:-gh, j, :], G.etot[gh:-gh, gh, :])
        assert np.array_equal(G.etot[gh:-gh, -1 - j, :], G.etot[gh:-gh, -gh - 1, :])


def test_sod_between_outflow_faces_matches_the_exact_solution(O):
    g = 1.4
    prm = O.params(gamma=g)
    N, gh = 100, 3
    x = (np.arange(N + 2 * gh) - gh + 0.5) / N
    shape = (1 + 2 * gh, 1 + 2 * gh, N + 2 * gh)
    rho = np.broadcast_to(np.where(x < 0.5, 1.0, 0.125), shape).copy()
    p = np.broadcast_to(np.where(x < 0.5, 1.0, 0.1), shape).copy()
    z = np.zeros(shape)
    st = W.stored_from_primitive(rho, z, z.copy(), z.copy(), p, g)
    d = dict(zip(O.FIELDS, [np.ascontiguousarray(a) for a in st]))
    G = O.Grid(**d, dx=1.0 / N, dy=1.0, dz=1.0, ghost=gh)
    t, s = 0.0, 0
    while t < 0.25 * (1 - 1e-14):
        O.fill_boundary(G, [O_, O_, P_, P_, P_, P_])
        dt = min(O.cfl_dt(G, prm), 0.25 - t)
        O.step(G, prm, dt, s % 2)
        t += dt
        s += 1
    r = G.rho[gh, gh, gh:-gh]
    rex, *_ = O.exact_riemann(g, [1.0, 0.0, 1.0], [0.125, 0.0, 0.1], (x[gh:-gh] - 0.5) / 0.25)
    e1 = np.sum(np.abs(r - rex)) / N
    assert e1 < 4e-3, e1


def test_uniform_inflow_to_outflow_stays_uniform(O):
    # a uniform flow entering at -x and leaving at +x is a steady solution
    g = 5.0 / 3.0
    prm = O.params(gamma=g)
    gh = 3
    shape = (4 + 2 * gh, 5 + 2 * gh, 12 + 2 * gh)
    st = W.stored_from_primitive(np.full(shape, 0.8), np.full(shape, 0.6), np.full(shape, -0.1),
                                 np.full(shape, 0.2), np.full(shape, 1.3), g)
    d = dict(zip(O.FIELDS, [np.ascontiguousarray(a) for a in st]))
    G = O.Grid(**_copy(d), dx=1.0 / 12, dy=1.0 / 5, dz=1.0 / 4, ghost=gh)
    inflow = np.zeros((6, 6))
    inflow[0] = [d[f].flat[0] for f in O.FIELDS]
    for s in range(4):
        O.fill_boundary(G, [I_, O_, P_, P_, P_, P_], inflow)
        O.step(G, prm, O.cfl_dt(G, prm), s % 2)
    act = (slice(gh, -gh),) * 3
    for f in O.FIELDS:
        a = getattr(G, f)[act]
        assert np.allclose(a, d[f].flat[0], rtol=1e-13, atol=1e-15), f
    # the inflow ghosts hold the given state
    assert np.array_equal(G.rho[gh:-gh, gh:-gh, :gh], np.full((4, 5, gh), inflow[0][0]))


def test_invalid_boundary_kinds_are_rejected(O):
    d = W.random_grid(4, 4, 2, 13, W.GENTLE)
    G = _grid(O, d)
    with pytest.raises(ValueError):
        O.fill_boundary(G, [P_, O_, P_, P_, P_, P_])      # unpaired periodic face
    with pytest.raises(ValueError):
        O.fill_boundary(G, [O_, O_, P_, P_, R_, R_])      # 2 active cells < 3 ghosts
    with pytest.raises(ValueError):
        O.fill_boundary(G, [I_, O_, P_, P_, P_, P_])      # inflow without values
    with pytest.raises(ValueError):
        O.fill_boundary(G, [7, O_, P_, P_, P_, P_])
