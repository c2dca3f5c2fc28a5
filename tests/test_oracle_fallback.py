"""Oracle pins of the positivity fallback (Sec. "Riemann Solvers and Fallback").

Two parts of the fallback are pinned here against something other than the
oracle itself:

* The HLL flux of a face inside the wave fan.  When the two outer wave speeds
  s_L <= s_R bound every wave of the exact Riemann solution, integral
  conservation over the space-time box [s_L t, s_R t] x [0, t] makes the
  average of the exact solution over the fan equal to
      U_bar = (s_R U_R - s_L U_L - (F_R - F_L)) / (s_R - s_L),
  and the HLL flux at x/t = 0 is the Rankine-Hugoniot flux across the left
  wave, F_L + s_L (U_bar - U_L).  U_bar is computed here by integrating the
  independent exact solver (Toro ch. 4) over the fan, so the subsonic HLL
  flux, and its face velocity (the velocity of the averaged state,
  U_bar_m / U_bar_rho), are pinned by the exact solution.  The internal
  energy is conserved only where no compression acts, so its component is
  checked on a moving contact.
* A cell still non-positive after the HLL re-solve: density raised to the
  floor with the old velocity kept, pressure set to the floor, counted once.
  A cell floored on its pressure alone keeps the momentum of its update,
  which the flux registers' telescoping pins (mass and momentum of the pencil
  change by the boundary fluxes only).
"""
from __future__ import annotations

import numpy as np
import pytest

G14 = 1.4


def _conserved(g, s):
    """Conserved vector and physical flux of a state (rho, u, v1, v2, p)."""
    r, u, v1, v2, p = s
    e = p / ((g - 1.0) * r)
    E = e + 0.5 * (u * u + v1 * v1 + v2 * v2)
    U = np.array([r, r * u, r * v1, r * v2, r * E, r * e])
    F = np.array([r * u, r * u * u + p, r * u * v1, r * u * v2, u * (r * E + p), r * u * e])
    return U, F


def _davis(g, sl, sr):
    cl = np.sqrt(g * sl[4] / sl[0])
    cr = np.sqrt(g * sr[4] / sr[0])
    return min(sl[1] - cl, sr[1] - cr), max(sl[1] + cl, sr[1] + cr)


def _exact_conserved(O, g, sl, sr, xi):
    """Exact solution at x/t = xi as conserved vectors [6, len(xi)]; the
    transverse velocities ride with the contact."""
    rho, u, p, star = O.exact_riemann(g, [sl[0], sl[1], sl[4]], [sr[0], sr[1], sr[4]], xi)
    left = xi < star["u_star"]
    v1 = np.where(left, sl[2], sr[2])
    v2 = np.where(left, sl[3], sr[3])
    e = p / ((g - 1.0) * rho)
    E = e + 0.5 * (u * u + v1 * v1 + v2 * v2)
    return np.array([rho, rho * u, rho * v1, rho * v2, rho * E, rho * e])


def _wave_edges(O, g, sl, sr):
    """Speeds at which the exact solution is not smooth: the contact, each
    shock, and the head and tail of each rarefaction (from the exact star
    state)."""
    _, _, _, st = O.exact_riemann(g, [sl[0], sl[1], sl[4]], [sr[0], sr[1], sr[4]], [0.0])
    ps, us = st["p_star"], st["u_star"]
    edges = [us]
    for s, rs, sgn in ((sl, st["rho_star_l"], -1.0), (sr, st["rho_star_r"], 1.0)):
        if ps > s[4]:  # shock: speed from the mass jump
            edges.append((rs * us - s[0] * s[1]) / (rs - s[0]))
        else:          # rarefaction: head and tail characteristics
            edges.append(s[1] + sgn * np.sqrt(g * s[4] / s[0]))
            edges.append(us + sgn * np.sqrt(g * ps / rs))
    return edges


def _fan_average(O, g, sl, sr, order=48):
    sL, sR = _davis(g, sl, sr)
    # every wave of the exact solution lies inside [sL, sR]
    UL, _ = _conserved(g, sl)
    UR, _ = _conserved(g, sr)
    out = _exact_conserved(O, g, sl, sr, np.array([sL - 1e-9, sR + 1e-9]))
    assert np.allclose(out[:, 0], UL, rtol=1e-13, atol=1e-14), "left wave outside the fan"
    assert np.allclose(out[:, 1], UR, rtol=1e-13, atol=1e-14), "right wave outside the fan"
    # Gauss-Legendre on each piece between the edges, where the solution is
    # constant or a smooth rarefaction fan
    cuts = sorted({sL, sR, *[min(max(w, sL), sR) for w in _wave_edges(O, g, sl, sr)]})
    x, w = np.polynomial.legendre.leggauss(order)
    total = np.zeros(6)
    for a, b in zip(cuts[:-1], cuts[1:]):
        if b > a:
            xi = 0.5 * (a + b) + 0.5 * (b - a) * x
            total += 0.5 * (b - a) * (_exact_conserved(O, g, sl, sr, xi) * w).sum(axis=1)
    return sL, sR, total / (sR - sL)


# (left, right) traced states (rho, u, v1, v2, p), all subsonic at the face
FAN_CASES = {
    # Sod-type: hot left gas, left rarefaction, contact, right shock
    "rarefaction-shock": ([1.0, 0.0, 0.3, -0.1, 10.0], [1.0, 0.0, -0.2, 0.4, 1.0]),
    # two rarefactions of unequal strength, flow through the face
    "double-rarefaction": ([1.0, -0.5, 0.1, 0.2, 1.0], [0.5, 0.8, -0.3, 0.0, 0.3]),
    # right-moving hot piston into a dense gas: left rarefaction, right shock
    "moving-shock": ([0.4, 0.6, 0.0, 0.5, 6.0], [1.2, 0.2, 0.7, -0.1, 1.5]),
}


@pytest.mark.parametrize("case", list(FAN_CASES))
def test_hll_flux_is_the_exact_fan_average(O, case):
    sl, sr = (np.array(s) for s in FAN_CASES[case])
    prm = O.params(gamma=G14)
    sL, sR, Ubar = _fan_average(O, G14, sl, sr)
    assert sL < 0.0 < sR  # a subsonic face: the fan branch of the solver
    UL, FL = _conserved(G14, sl)
    _, FR = _conserved(G14, sr)
    want = FL + sL * (Ubar - UL)
    got = O.hll_flux(prm, sl, sr)
    scale = np.maximum(np.maximum(np.abs(FL), np.abs(FR)), 1.0)
    # mass, momentum and total energy are conserved by the exact solution
    err = np.abs(got[:5] - want[:5]) / scale[:5]
    assert err.max() < 1e-12, (got[:5], want[:5], err)
    # face velocity of the p div v term: that of the averaged state
    assert got[6] == pytest.approx(Ubar[1] / Ubar[0], rel=1e-12, abs=1e-13)


def test_hll_internal_energy_flux_on_a_moving_contact(O):
    # no compression anywhere: rho e is conserved and obeys the same identity
    sl = np.array([1.0, 0.4, 0.2, -0.3, 1.0])
    sr = np.array([0.2, 0.4, -0.5, 0.1, 1.0])
    prm = O.params(gamma=G14)
    sL, sR, Ubar = _fan_average(O, G14, sl, sr)
    UL, FL = _conserved(G14, sl)
    want = FL + sL * (Ubar - UL)
    got = O.hll_flux(prm, sl, sr)
    scale = np.maximum(np.abs(FL), 1.0)
    err = np.abs(got[:6] - want) / scale
    assert err.max() < 1e-12, (got[:6], want, err)
    assert got[6] == pytest.approx(0.4, rel=1e-12)


def _diverging_pencil(g, U, p0, n=20):
    """Uniform gas with one cell (moving at 0.05) between two cells flowing
    away from it at speed U; transverse velocities 0.3 and -0.2."""
    c = n // 2
    rho = np.ones(n)
    p = np.full(n, p0)
    u = np.zeros(n)
    u[c - 1], u[c], u[c + 1] = -U, 0.05, U
    v1 = np.full(n, 0.3)
    v2 = np.full(n, -0.2)
    e = p / ((g - 1.0) * rho)
    E = e + 0.5 * (u * u + v1 * v1 + v2 * v2)
    return [a.copy() for a in (rho, u, v1, v2, E, e)], c


def test_cell_floored_on_density_keeps_its_old_velocity(O):
    g = 5.0 / 3.0
    prm = O.params(gamma=g)
    arr, c = _diverging_pencil(g, U=4.0, p0=0.01)
    old = [a.copy() for a in arr]
    cnt, _, _ = O.pencil(prm, 0.2, 1.0, *arr)
    rho, u, v1, v2, E, e = arr
    # the centre cell empties under both two-shock and HLL fluxes
    assert cnt.floored_cells == 1 and cnt.fallback_faces == 2
    assert rho[c] == prm.rho_floor
    assert (u[c], v1[c], v2[c]) == (old[1][c], old[2][c], old[3][c])
    # its pressure is the floor: p = (g - 1) rho e
    assert (g - 1.0) * rho[c] * e[c] == pytest.approx(prm.p_floor, rel=1e-15, abs=0.0)
    assert E[c] == pytest.approx(e[c] + 0.5 * (u[c] ** 2 + v1[c] ** 2 + v2[c] ** 2), rel=1e-15)
    # every other active cell stays physical
    others = [j for j in range(3, len(rho) - 3) if j != c]
    assert np.all(rho[others] > prm.rho_floor) and np.all(e[others] > 0.0)


def test_cell_floored_on_pressure_keeps_the_momentum_of_its_update(O):
    g = 5.0 / 3.0
    prm = O.params(gamma=g)
    arr, c = _diverging_pencil(g, U=4.0, p0=1.0)
    old = [a.copy() for a in arr]
    dt, dx = 0.2, 1.0
    cnt, lo, hi = O.pencil(prm, dt, dx, *arr, want_reg=True)
    rho, u, v1, v2, E, e = arr
    assert cnt.floored_cells == 1 and cnt.fallback_faces == 2
    assert rho[c] > prm.rho_floor and u[c] != old[1][c]
    assert (g - 1.0) * rho[c] * e[c] == pytest.approx(prm.p_floor, rel=1e-15, abs=0.0)
    assert E[c] == pytest.approx(e[c] + 0.5 * (u[c] ** 2 + v1[c] ** 2 + v2[c] ** 2), rel=1e-15)
    # mass and the three momenta change by the boundary fluxes alone (the
    # registers hold dt F of the first and last active faces)
    act = slice(3, len(rho) - 3)
    for k, (new_q, old_q) in enumerate([(rho, old[0]),
                                        (rho * u, old[0] * old[1]),
                                        (rho * v1, old[0] * old[2]),
                                        (rho * v2, old[0] * old[3])]):
        change = new_q[act].sum() - old_q[act].sum()
        assert change == pytest.approx(-(hi[k] - lo[k]) / dx, abs=1e-13), k
