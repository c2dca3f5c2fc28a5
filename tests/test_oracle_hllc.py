"""Pins of the oracle's HLLC solver (CPU only).

HLLC is the three-wave approximate Riemann solver the paper lists beside
two-shock and HLL (Sec. "Riemann Solvers and Fallback"); the oracle selects it
with the HLLC flag.  The pins do not retype its formulas: they check the
Rankine-Hugoniot conditions across its outer waves and its contact (a
common pressure and normal velocity on both sides of the contact), exact
treatment of isolated contacts (the property that separates it from HLL),
consistency, upwinding, mirror symmetry, and the whole PPM sweep with HLLC
against the exact Sod solution and the invariants of the scheme.
"""
import numpy as np
import pytest

from paper_1307_2265_amd import workloads as W
from tests.test_oracle_sweeps import G3, _evolve_1d, _grid

G = 1.4


def _phys(g, s):
    """Euler flux of a state (rho, u, v1, v2, p): F_rho, F_u, F_v1, F_v2, F_E, F_e."""
    rho, u, v1, v2, p = s
    e = p / ((g - 1) * rho)
    E = e + 0.5 * (u * u + v1 * v1 + v2 * v2)
    return np.array([rho * u, rho * u * u + p, rho * u * v1, rho * u * v2, u * (rho * E + p),
                     rho * u * e])


def _cons(g, s):
    rho, u, v1, v2, p = s
    e = p / ((g - 1) * rho)
    E = e + 0.5 * (u * u + v1 * v1 + v2 * v2)
    return np.array([rho, rho * u, rho * v1, rho * v2, rho * E, rho * e])


def _davis(g, L, R):
    cl, cr = np.sqrt(g * L[4] / L[0]), np.sqrt(g * R[4] / R[0])
    return min(L[1] - cl, R[1] - cr), max(L[1] + cl, R[1] + cr)


SUBSONIC = [
    ([1.0, 0.0, 0.0, 0.0, 1.0], [0.125, 0.0, 0.0, 0.0, 0.1]),      # Sod
    ([1.0, 0.75, 0.1, -0.2, 1.0], [0.125, 0.0, 0.3, 0.0, 0.1]),    # Toro test 1 + shear
    ([1.0, -2.0, 0.0, 0.5, 0.4], [1.0, 2.0, 0.0, 0.5, 0.4]),       # double rarefaction
    ([5.99924, 19.5975, 0.0, 0.0, 460.894], [5.99242, -6.19633, 1.0, 0.0, 46.0950]),
    ([0.7, 0.2, 0.0, 0.0, 2.0], [1.3, -0.4, 0.0, -0.3, 0.5]),
]


@pytest.mark.parametrize("L,R", SUBSONIC)
def test_hllc_flux_satisfies_the_jump_conditions_of_its_waves(O, L, R):
    # Inside the fan the flux is that of a star state U*_K reached from U_K
    # across the outer wave s_K (F* - F_K = s_K (U* - U_K)) and carrying the
    # contact's common pressure and normal velocity S*: so F*_rho = rho* S*,
    # F*_u = rho* S*^2 + p*, F*_E = S* (rho* E* + p*), and p* is the same
    # whether it is derived from the left or the right data.
    prm = O.params(gamma=G)
    L, R = np.array(L), np.array(R)
    f = O.hllc_flux(prm, L, R)
    S = f[6]
    sL, sR = _davis(G, L, R)
    assert sL < 0.0 < sR
    pstar = {}
    for side, st, s in (("L", L, sL), ("R", R, sR)):
        U, F = _cons(G, st), _phys(G, st)
        # the star state from the mass and momentum jump conditions and the
        # contact velocity: rho* (s - S*) = rho (s - u)
        rs = st[0] * (s - st[1]) / (s - S)
        ps = F[1] + s * (rs * S - U[1]) - rs * S * S
        Es = (s * U[4] - F[4] + S * ps) / (s - S)
        pstar[side] = (ps, rs, Es)
    assert pstar["L"][0] == pytest.approx(pstar["R"][0], rel=1e-12)
    K = "L" if S >= 0 else "R"
    ps, rs, Es = pstar[K]
    scale = np.abs(f[:6]).max()
    assert abs(f[0] - rs * S) <= 1e-13 * scale
    assert abs(f[1] - (rs * S * S + ps)) <= 1e-13 * scale
    assert abs(f[4] - S * (Es + ps)) <= 1e-13 * scale
    # transverse velocities and internal energy ride with the mass flux
    st = L if K == "L" else R
    assert f[2] == pytest.approx(f[0] * st[2], rel=1e-13, abs=1e-15 * scale)
    assert f[3] == pytest.approx(f[0] * st[3], rel=1e-13, abs=1e-15 * scale)
    assert f[5] == pytest.approx(f[0] * st[4] / ((G - 1) * st[0]), rel=1e-13, abs=1e-15 * scale)


def test_hllc_star_state_tends_to_the_exact_one_for_weak_waves(O):
    # The outer wave speeds u -+ c are exact for acoustic waves, so the HLLC
    # contact velocity and pressure approach the exact Riemann solution's at
    # second order in the jump size.
    prm = O.params(gamma=G)
    errs = []
    for d in (1e-2, 1e-3):
        L = [1.0, 0.1, 0.0, 0.0, 1.0]
        R = [1.0 - d, 0.1 + 0.4 * d, 0.0, 0.0, 1.0 - 1.3 * d]
        f = O.hllc_flux(prm, np.array(L), np.array(R))
        *_, star = O.exact_riemann(G, [L[0], L[1], L[4]], [R[0], R[1], R[4]], [0.0])
        errs.append(max(abs(f[6] - star["u_star"]),
                        abs((f[1] - f[6] * f[0]) - star["p_star"])))
    assert errs[0] < 1e-4, errs
    assert errs[0] / errs[1] > 50, errs


@pytest.mark.parametrize("u", [0.0, 0.3, -0.45])
def test_hllc_resolves_an_isolated_contact_exactly(O, u):
    # Equal pressure and normal velocity, a density jump and sheared
    # transverse velocities: the exact flux is the upwind physical flux
    # (zero mass flux for a stationary contact).  HLL smears it.
    prm = O.params(gamma=G)
    L = np.array([1.0, u, 0.2, -0.1, 1.0])
    R = np.array([0.125, u, 0.5, 0.7, 1.0])
    f = O.hllc_flux(prm, L, R)
    up = _phys(G, L if u >= 0 else R)
    scale = np.abs(up).max()
    assert np.max(np.abs(f[:6] - up)) <= 1e-14 * scale
    assert f[6] == pytest.approx(u, abs=1e-15)
    if u == 0.0:
        assert f[0] == 0.0 and f[4] == 0.0 and f[1] == 1.0
    h = O.hll_flux(prm, L, R)
    assert np.max(np.abs(h[:6] - up)) > 1e-2 * scale


@pytest.mark.parametrize("s", [[0.8, 0.3, -0.2, 0.1, 1.3], [1.0, 5.0, 0.0, 0.0, 1.0],
                               [1.0, -5.0, 0.3, 0.0, 1.0], [0.5, 0.0, 0.0, 0.0, 2.0]])
def test_hllc_is_consistent(O, s):
    prm = O.params(gamma=G)
    s = np.array(s)
    f = O.hllc_flux(prm, s, s)
    phys = _phys(G, s)
    assert np.allclose(f[:6], phys, rtol=1e-14, atol=1e-15)
    assert f[6] == pytest.approx(s[1], rel=1e-14, abs=1e-15)


def test_hllc_upwinds_supersonic_states_like_hll(O):
    prm = O.params(gamma=G)
    fast = np.array([1.0, 5.0, 0.2, 0.0, 1.0])
    other = np.array([0.1, 5.0, 0.0, 0.3, 0.1])
    assert np.array_equal(O.hllc_flux(prm, fast, other), O.hll_flux(prm, fast, other))
    assert np.array_equal(O.hllc_flux(prm, fast, other)[:6], _phys(G, fast))
    back = np.array([1.0, -5.0, 0.2, 0.0, 1.0])
    assert np.array_equal(O.hllc_flux(prm, other * [1, -1, 1, 1, 1], back),
                          O.hll_flux(prm, other * [1, -1, 1, 1, 1], back))


@pytest.mark.parametrize("L,R", SUBSONIC)
def test_hllc_mirror_symmetry(O, L, R):
    # Reflecting x -> -x swaps the states and negates normal velocities: the
    # mass, transverse-momentum, energy fluxes and the face velocity change
    # sign, the normal-momentum flux does not.
    prm = O.params(gamma=G)
    L, R = np.array(L), np.array(R)
    m = np.array([1, -1, 1, 1, 1])
    f = O.hllc_flux(prm, L, R)
    g = O.hllc_flux(prm, R * m, L * m)
    sign = np.array([-1, 1, -1, -1, -1, -1, -1])
    assert np.allclose(g, sign * f, rtol=1e-14, atol=1e-14 * np.abs(f).max())


def _sod_E1_hllc(O, N):
    prm = O.params(gamma=G, flags=O.ALL_FLAGS | O.HLLC)
    dx = 1.0 / N
    x = (np.arange(N + 6) - G3 + 0.5) * dx
    rho = np.where(x < 0.5, 1.0, 0.125)
    p = np.where(x < 0.5, 1.0, 0.1)
    r, *_ = _evolve_1d(O, prm, rho, np.zeros_like(x), p, dx, 0.25)
    xa = x[G3:-G3]
    rex, *_ = O.exact_riemann(G, [1.0, 0.0, 1.0], [0.125, 0.0, 0.1], (xa - 0.5) / 0.25)
    return np.sum(dx * np.abs(r[G3:-G3] - rex)), r[G3:-G3]


def test_ppm_with_hllc_converges_to_the_exact_sod_solution(O):
    e100, r100 = _sod_E1_hllc(O, 100)
    e200, _ = _sod_E1_hllc(O, 200)
    assert e100 < 4e-3, e100
    assert e200 / e100 < 0.7, (e100, e200)
    assert r100.min() > 0.125 - 1e-9 and r100.max() < 1.0 + 1e-9


def test_ppm_with_hllc_keeps_a_stationary_contact(O):
    # A density jump at rest in uniform pressure is a steady solution; with
    # HLLC the mass flux through it vanishes, so velocity stays zero and the
    # density profile and pressure stay as they were, to round-off.
    prm = O.params(gamma=G, flags=O.ALL_FLAGS | O.HLLC)
    N = 64
    dx = 1.0 / N
    x = (np.arange(N + 6) - G3 + 0.5) * dx
    rho = np.where(np.abs(x - 0.5) < 0.2, 1.0, 0.125)
    p = np.ones_like(x)
    r, u, pp, *_ = _evolve_1d(O, prm, rho, np.zeros_like(x), p, dx, 0.3, bc="periodic",
                              v1=np.sin(2 * np.pi * x))
    assert np.max(np.abs(u[G3:-G3])) <= 1e-13
    assert np.max(np.abs(pp[G3:-G3] - 1.0)) <= 1e-13
    assert np.max(np.abs(r[G3:-G3] - rho[G3:-G3])) <= 1e-13


@pytest.mark.parametrize("recipe,flatten,ghost", [(W.GENTLE, False, 3), (W.SHOCKED, True, 4)])
def test_hllc_sweeps_conserve_in_a_periodic_box(O, recipe, flatten, ghost):
    # as for two-shock: fluxes telescope (a fourth ghost layer where the
    # flattening of the outermost reconstructed cell would differ between the
    # two periodic images of the boundary face)
    prm = O.params(flags=(O.ALL_FLAGS if flatten else O.ALL_FLAGS & ~O.FLATTEN) | O.HLLC)
    d = W.random_grid(20, 16, 12, 77, recipe, ghost=ghost)
    Gr = _grid(O, d, ghost=ghost)
    sl = (slice(ghost, -ghost),) * 3
    for s in range(3):
        O.fill_periodic(Gr)
        dt = O.cfl_dt(Gr, prm)
        m0 = [Gr.rho[sl], Gr.rho[sl] * Gr.vx[sl], Gr.rho[sl] * Gr.vy[sl], Gr.rho[sl] * Gr.vz[sl],
              Gr.rho[sl] * Gr.etot[sl]]
        tot0 = [m.sum() for m in m0]
        scale = [np.abs(m).sum() for m in m0]
        c = O.step(Gr, prm, dt, s % 2)
        assert c.floored_cells == 0
        m1 = [Gr.rho[sl], Gr.rho[sl] * Gr.vx[sl], Gr.rho[sl] * Gr.vy[sl], Gr.rho[sl] * Gr.vz[sl],
              Gr.rho[sl] * Gr.etot[sl]]
        for a, b, sc in zip(m1, tot0, scale):
            assert abs(a.sum() - b) <= 64 * np.finfo(float).eps * sc


def test_hllc_and_two_shock_agree_on_smooth_flow(O):
    # Same reconstruction, different solver: on a smooth, well-resolved wave
    # the face jumps are small and both solvers give the exact linearised
    # flux, so one step agrees to second order in the wave amplitude; they
    # are not the same scheme, so the results are not identical.
    g = 5.0 / 3.0
    n = 16
    x = (np.arange(n + 2 * G3) - G3 + 0.5) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    ph = 2 * np.pi * (X + 2 * Y + Z)
    diffs = []
    for amp in (1e-2, 1e-3):
        st = W.stored_from_primitive(1.0 + amp * np.sin(ph), amp * np.cos(ph),
                                     0.5 * amp * np.sin(ph), np.zeros_like(X),
                                     1.0 + amp * np.cos(ph + 0.3), g)
        d = dict(zip(O.FIELDS, [np.ascontiguousarray(a) for a in st]))
        out = {}
        for name, extra in (("ts", 0), ("hllc", O.HLLC)):
            prm = O.params(gamma=g, flags=O.ALL_FLAGS | extra)
            Gr = _grid(O, {k: v.copy() for k, v in d.items()})
            O.fill_periodic(Gr)
            O.step(Gr, prm, 0.5 * O.cfl_dt(Gr, prm), 0)
            out[name] = Gr.rho[(slice(G3, -G3),) * 3].copy()
        diffs.append(np.max(np.abs(out["ts"] - out["hllc"])))
    assert 0.0 < diffs[1] < 1e-9, diffs
    assert diffs[0] / diffs[1] > 50, diffs


@pytest.mark.parametrize("v,p0,dt", [(4.0, 0.4, 0.0015), (20.0, 0.01, 0.0004)])
def test_hllc_keeps_vacuum_forming_rarefactions_positive(O, v, p0, dt):
    # HLL-type fluxes with outer speeds that bound the waves keep density and
    # pressure positive; on a double rarefaction strong enough that the
    # two-shock update goes non-positive (and needs the HLL fallback), HLLC
    # needs no fallback.
    from tests.helpers import FIELDS, oracle_grid
    nx, ny, nz = 4, 100, 3
    shape = (nz + 6, ny + 6, nx + 6)
    y = (np.arange(ny + 6) - G3 + 0.5) / ny
    vy = np.broadcast_to(np.where(y < 0.5, -v, v)[None, :, None], shape).copy()
    z = np.zeros(shape)
    st = W.stored_from_primitive(np.ones(shape), z, vy, z.copy(), np.full(shape, p0), G)
    d = dict(zip(FIELDS, [np.ascontiguousarray(a) for a in st]))
    counts = {}
    for name, fl in (("two-shock", O.ALL_FLAGS), ("hllc", O.ALL_FLAGS | O.HLLC)):
        Gr = oracle_grid(O, d, dx=(0.25, 0.01, 1.0 / 3.0))
        prm = O.params(gamma=G, flags=fl)
        tot = [0, 0]
        for _ in range(16):
            c = O.step(Gr, prm, dt, 0)
            tot[0] += c.fallback_faces
            tot[1] += c.floored_cells
        counts[name] = tot
        if name == "hllc":
            assert np.all(Gr.rho > 0) and np.all(Gr.eint > 0)
    assert counts["two-shock"][0] > 0, counts
    assert counts["hllc"] == [0, 0], counts
