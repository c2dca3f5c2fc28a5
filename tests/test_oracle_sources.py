"""Pins of the oracle's gravity and comoving-expansion terms (CPU only).

The comoving equations (Sec. "Physical Equations") divide the flux
divergences by the expansion factor a, add the gravitational source rho g / a
to momentum and rho v g / a to total energy (time-centred as in Eqs.
momentum_diff and energy_diff, with the supplied acceleration at the half
step), and carry expansion terms that are split off and solved implicitly and
time-centred (Sec. "Hydrodynamics: The PPM method").  Pins: a uniform
medium in a uniform field accelerates exactly as v0 + n dt g / a with its
internal energy untouched; in a periodic box the total momentum grows by
exactly dt g M / a per step; with constant a the update is that of the static
equations with the time rescaled (a step of a dt with factor a equals a step
of dt with a = 1, bit for bit); the expansion terms converge at second order
to the exact decay of their ODEs; a zero field changes nothing.
"""
import numpy as np
import pytest

from paper_1307_2265_amd import workloads as W
from tests.test_oracle_sweeps import _grid

G3 = 3


def _uniform(nx, ny, nz, rho, v, p, gamma=5.0 / 3.0):
    return W.uniform_grid(nx, ny, nz, rho, v, p, gamma=gamma)


def _accel(shape, g):
    return tuple(np.full(shape, float(c)) for c in g)


@pytest.mark.parametrize("a", [1.0, 2.5])
def test_uniform_medium_accelerates_at_g_over_a(O, a):
    d = _uniform(8, 6, 5, 1.3, (0.2, -0.1, 0.05), 0.9)
    G = _grid(O, d)
    gvec = (0.7, -0.3, 0.2)
    G.accel = _accel(G.rho.shape, gvec)
    prm = O.params(a=a)
    e0 = G.eint.copy()
    dt, n = 1e-3, 6
    for s in range(n):
        O.fill_periodic(G)
        O.step(G, prm, dt, s % 2)
    act = (slice(G3, -G3),) * 3
    for v, v0, gc in zip((G.vx, G.vy, G.vz), (0.2, -0.1, 0.05), gvec):
        assert np.allclose(v[act], v0 + n * dt * gc / a, rtol=1e-13, atol=1e-15)
    assert np.allclose(G.rho[act], 1.3, rtol=1e-14)
    assert np.allclose(G.eint[act], e0[act], rtol=1e-13)
    # the gravitational work went into kinetic energy only
    ke = 0.5 * (G.vx ** 2 + G.vy ** 2 + G.vz ** 2)
    assert np.allclose(G.etot[act] - ke[act], G.eint[act], rtol=1e-12)


def test_momentum_grows_by_g_times_mass_in_a_periodic_box(O):
    # (four ghost layers: with three, flattening next to the periodic faces
    # makes the two images of a boundary face disagree, see the conservation pin)
    a, gh = 1.7, 4
    prm = O.params(a=a)
    d = W.random_grid(12, 10, 8, 61, W.GENTLE, ghost=gh)
    G = _grid(O, d, ghost=gh)
    gvec = (0.4, -0.25, 0.15)
    G.accel = _accel(G.rho.shape, gvec)
    act = (slice(gh, -gh),) * 3
    vol = G.dx * G.dy * G.dz
    for s in range(3):
        O.fill_periodic(G)
        dt = O.cfl_dt(G, prm)
        mass = G.rho[act].sum() * vol
        mom0 = [(G.rho * v)[act].sum() * vol for v in (G.vx, G.vy, G.vz)]
        c = O.step(G, prm, dt, s % 2)
        assert c.floored_cells == 0
        mom1 = [(G.rho * v)[act].sum() * vol for v in (G.vx, G.vy, G.vz)]
        assert G.rho[act].sum() * vol == pytest.approx(mass, rel=1e-13)
        for m0, m1, gc in zip(mom0, mom1, gvec):
            scale = (np.abs(G.rho * G.vx)[act].sum() + mass * abs(gc) * dt / a) * vol
            assert abs((m1 - m0) - dt * gc * mass / a) <= 1e-12 * scale


def test_constant_expansion_factor_rescales_time(O):
    # d/dt + (1/a) d/dx with constant a is the static system in t/a: a step of
    # a*dt with factor a is a step of dt with a = 1, and the gravity term
    # (dt/2)(g/a) is the same product too
    a = 2.0
    d = W.random_grid(10, 8, 6, 62, W.SHOCKED)
    A, B = _grid(O, {k: v.copy() for k, v in d.items()}), _grid(O, {k: v.copy() for k, v in d.items()})
    rng = np.random.default_rng(3)
    acc = tuple(rng.normal(size=A.rho.shape) for _ in range(3))
    A.accel, B.accel = acc, tuple(x.copy() for x in acc)
    pa, pb = O.params(a=a), O.params(a=1.0)
    for s in range(3):
        O.fill_periodic(A)
        O.fill_periodic(B)
        dt = O.cfl_dt(B, pb)
        assert O.cfl_dt(A, pa) == a * dt
        O.step(A, pa, a * dt, s % 2)
        O.step(B, pb, dt, s % 2)
    for f in O.FIELDS:
        assert np.array_equal(getattr(A, f), getattr(B, f)), f


def test_zero_field_changes_nothing(O):
    d = W.random_grid(9, 7, 6, 63, W.SHOCKED)
    A, B = _grid(O, {k: v.copy() for k, v in d.items()}), _grid(O, {k: v.copy() for k, v in d.items()})
    B.accel = _accel(B.rho.shape, (0.0, 0.0, 0.0))
    prm = O.params()
    for s in range(2):
        O.fill_periodic(A)
        O.fill_periodic(B)
        dt = O.cfl_dt(A, prm)
        O.step(A, prm, dt, s % 2)
        O.step(B, prm, dt, s % 2)
    for f in O.FIELDS:
        assert np.array_equal(getattr(A, f), getattr(B, f)), f


def test_expansion_terms_converge_at_second_order(O):
    # uniform state: dv/dt = -H v, d(rho E)/dt = -2 H rho E,
    # de/dt = -3 (gamma - 1) H e with H = adot / a held over the interval
    gamma = 5.0 / 3.0
    a, adot, T = 1.3, 0.9, 0.4
    H = adot / a
    errs = []
    for n in (10, 20, 40):
        d = _uniform(4, 4, 4, 1.0, (0.5, -0.2, 0.1), 1.0, gamma)
        G = _grid(O, d)
        v0, E0, e0 = G.vx.flat[0], G.etot.flat[0], G.eint.flat[0]
        prm = O.params(gamma=gamma, a=a, adot=adot)
        for _ in range(n):
            O.expansion(G, prm, T / n)
        c = (G3, G3, G3)
        errs.append(max(abs(G.vx[c] - v0 * np.exp(-H * T)) / abs(v0),
                        abs(G.etot[c] - E0 * np.exp(-2 * H * T)) / E0,
                        abs(G.eint[c] - e0 * np.exp(-3 * (gamma - 1) * H * T)) / e0))
    assert errs[0] < 1e-3, errs
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs
    # ghost cells are not touched
    assert G.vx[0, 0, 0] == v0
