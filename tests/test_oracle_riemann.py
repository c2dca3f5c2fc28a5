"""Pins of the oracle's Riemann solvers (CPU only).

The exact solver is pinned by the textbook Sod star state and by the jump
conditions its solution must satisfy (Rankine-Hugoniot across shocks,
isentropy and the Riemann invariant across rarefactions, continuity of p and
u across the contact).  The two-shock solver (paper Sec. "Riemann Solvers and
Fallback": both waves treated as shocks, pressure found iteratively) is exact
whenever both waves really are shocks, so it is pinned against the exact
solver there, and by its symmetries elsewhere.
"""
import numpy as np
import pytest

from tests.golden.load import load


def _exact_star(O, g, L, R):
    return O.exact_riemann(g, L, R, [0.0])[3]


def test_exact_sod_star_state_matches_textbook(O):
    d = load("sod_star_state.txt")
    star = _exact_star(O, d["gamma"], [d["rho_L"], d["u_L"], d["p_L"]],
                       [d["rho_R"], d["u_R"], d["p_R"]])
    # the reference is printed to 5 significant figures
    assert star["p_star"] == pytest.approx(d["p_star"], abs=5e-6)
    assert star["u_star"] == pytest.approx(d["u_star"], abs=5e-6)
    assert star["rho_star_l"] == pytest.approx(d["rho_star_L"], abs=5e-6)
    assert star["rho_star_r"] == pytest.approx(d["rho_star_R"], abs=5e-6)


def _shock_jump_residuals(g, pre, post, S):
    """Mass, momentum and energy flux continuity in the frame of a shock of speed S."""
    def flux(rho, u, p):
        w = u - S
        E = p / (g - 1.0) + 0.5 * rho * u * u
        return np.array([rho * w, rho * u * w + p, E * w + p * u])
    # F(U) - S U is continuous: F_pre - S U_pre == F_post - S U_post
    f_pre, f_post = flux(*pre), flux(*post)
    return np.abs(f_pre - f_post) / (1.0 + np.abs(f_pre))


@pytest.mark.parametrize("L,R,g", [
    ([1.0, 0.0, 1.0], [0.125, 0.0, 0.1], 1.4),       # Sod: rarefaction + shock
    ([1.0, 0.75, 1.0], [0.125, 0.0, 0.1], 1.4),
    ([5.99924, 19.5975, 460.894], [5.99242, -6.19633, 46.095], 1.4),  # two shocks
    ([1.0, -1.0, 0.4], [1.0, 1.0, 0.4], 5.0 / 3.0),  # two rarefactions
])
def test_exact_solution_satisfies_jump_conditions(O, L, R, g):
    rho_s, u_s, p_s, star = O.exact_riemann(g, L, R, [0.0])
    ps, us = star["p_star"], star["u_star"]
    for side, rs, sgn in ((L, star["rho_star_l"], -1.0), (R, star["rho_star_r"], 1.0)):
        rho, u, p = side
        c = np.sqrt(g * p / rho)
        if ps > p:
            # shock: speed from mass conservation, then all three jumps must hold
            S = (rs * us - rho * u) / (rs - rho)
            res = _shock_jump_residuals(g, (rho, u, p), (rs, us, ps), S)
            assert np.all(res < 1e-12), res
            assert sgn * (S - u) > 0.0  # the shock moves away from the contact
        else:
            # rarefaction: isentropic, and the Riemann invariant across it is constant
            assert ps / rs**g == pytest.approx(p / rho**g, rel=1e-12)
            cs = np.sqrt(g * ps / rs)
            inv = u - sgn * 2.0 * c / (g - 1.0)
            inv_s = us - sgn * 2.0 * cs / (g - 1.0)
            assert inv_s == pytest.approx(inv, rel=1e-12, abs=1e-12)


def test_exact_rarefaction_fan_is_self_similar(O):
    g = 1.4
    L, R = [1.0, 0.0, 1.0], [0.125, 0.0, 0.1]
    xi = np.linspace(-1.1, -0.1, 41)  # inside and around the left fan
    rho, u, p, star = O.exact_riemann(g, L, R, xi)
    c = np.sqrt(g * p / rho)
    head = -np.sqrt(g)
    fan = (xi > head) & (xi < star["u_star"] - np.sqrt(g * star["p_star"] / star["rho_star_l"]))
    assert fan.sum() > 10
    # inside a left-facing centred fan the C- characteristic is x/t: u - c = xi
    assert np.allclose((u - c)[fan], xi[fan], rtol=0, atol=1e-12)
    assert np.allclose(p[fan] / rho[fan]**g, 1.0, rtol=1e-12)


@pytest.mark.parametrize("L,R,g", [
    ([1.0, 2.0, 1.0], [1.0, -2.0, 1.0], 5.0 / 3.0),
    ([1.0, 2.0, 1.0], [0.5, -1.0, 3.0], 5.0 / 3.0),
    ([5.99924, 19.5975, 460.894], [5.99242, -6.19633, 46.095], 1.4),
    ([0.3, 10.0, 0.01], [2.0, 0.0, 0.02], 1.4),
    ([1.0, 2.5, 10.0], [3.0, -2.5, 2.0], 1.1),
])
def test_two_shock_exact_when_both_waves_are_shocks(O, L, R, g):
    star = _exact_star(O, g, L, R)
    assert star["p_star"] > max(L[2], R[2])  # both waves are shocks
    prm = O.params(gamma=g)
    ts = O.two_shock(prm, L, R)
    assert ts["p_star"] == pytest.approx(star["p_star"], rel=1e-12)
    assert ts["u_star"] == pytest.approx(star["u_star"], rel=1e-12, abs=1e-12)
    rho, u, p, _ = O.exact_riemann(g, L, R, [0.0])
    assert ts["rho"] == pytest.approx(rho[0], rel=1e-11)
    assert ts["u"] == pytest.approx(u[0], rel=1e-11, abs=1e-12)
    assert ts["p"] == pytest.approx(p[0], rel=1e-11)


def test_two_shock_mirror_symmetry(O):
    rng = np.random.default_rng(5)
    prm = O.params(gamma=5.0 / 3.0)
    for _ in range(200):
        L = [rng.lognormal(0, 1), rng.normal(0, 2), rng.lognormal(0, 1)]
        R = [rng.lognormal(0, 1), rng.normal(0, 2), rng.lognormal(0, 1)]
        a = O.two_shock(prm, L, R)
        b = O.two_shock(prm, [R[0], -R[1], R[2]], [L[0], -L[1], L[2]])
        assert a["p_star"] == b["p_star"]
        assert a["u_star"] == -b["u_star"]
        # the sampled flux-relevant state mirrors too (except the side chosen at u* = 0)
        if a["u_star"] != 0.0:
            assert a["rho"] == b["rho"] and a["p"] == b["p"] and a["u"] == -b["u"]


def test_two_shock_contact_and_uniform(O):
    prm = O.params(gamma=1.4)
    ts = O.two_shock(prm, [1.0, 0.3, 2.0], [0.1, 0.3, 2.0])  # pure contact
    assert ts["p_star"] == pytest.approx(2.0, rel=1e-15)
    assert ts["u_star"] == pytest.approx(0.3, rel=1e-15)
    assert ts["rho"] == pytest.approx(1.0, rel=1e-14)  # upwind (left) density
    ts = O.two_shock(prm, [0.7, -0.2, 1.5], [0.7, -0.2, 1.5])
    assert ts["p_star"] == pytest.approx(1.5, rel=1e-15) and not ts["left"]


def test_two_shock_weak_waves_agree_with_exact_to_second_order(O):
    # For a rarefaction the two-shock pressure differs from the exact one at
    # third order in the wave strength (shock and rarefaction curves osculate).
    g = 1.4
    prm = O.params(gamma=g)
    errs = []
    for eps in (0.1, 0.05, 0.025):
        L, R = [1.0, 0.0, 1.0], [1.0, eps, 1.0]  # two weak rarefactions
        ts = O.two_shock(prm, L, R)
        star = _exact_star(O, g, L, R)
        errs.append(abs(ts["p_star"] - star["p_star"]))
    order = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    assert min(order) > 2.7, (errs, order)


def test_two_shock_converges_within_iteration_cap(O):
    rng = np.random.default_rng(9)
    prm = O.params(gamma=5.0 / 3.0)
    for _ in range(500):
        L = [rng.lognormal(0, 2), rng.normal(0, 6), rng.lognormal(0, 1)]
        R = [rng.lognormal(0, 2), rng.normal(0, 6), rng.lognormal(0, 1)]
        ts = O.two_shock(prm, L, R)
        assert ts["iters"] < 20 and ts["p_star"] > 0.0 and np.isfinite(ts["u_star"])


def test_hll_flux_consistency_and_upwinding(O):
    g = 1.4
    prm = O.params(gamma=g)
    s = np.array([0.8, 0.3, -0.2, 0.1, 1.3])  # rho,u,v1,v2,p
    rho, u, v1, v2, p = s
    e = p / ((g - 1) * rho)
    E = e + 0.5 * (u * u + v1 * v1 + v2 * v2)
    phys = np.array([rho * u, rho * u * u + p, rho * u * v1, rho * u * v2, u * (rho * E + p),
                     rho * u * e])
    f = O.hll_flux(prm, s, s)
    assert np.allclose(f[:6], phys, rtol=1e-14, atol=1e-15)  # F(U, U) = F(U)
    assert f[6] == pytest.approx(u, rel=1e-14)
    sup = np.array([1.0, 5.0, 0.0, 0.0, 1.0])  # supersonic to the right: left flux
    other = np.array([0.1, 5.0, 0.0, 0.0, 0.1])
    assert np.array_equal(O.hll_flux(prm, sup, other)[:6], O.hll_flux(prm, sup, sup)[:6])
