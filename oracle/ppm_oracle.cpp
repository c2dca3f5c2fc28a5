// ppm_oracle.cpp -- TEST INFRASTRUCTURE ONLY (see ppm_oracle.h).
//
// A deliberately plain FP64 implementation of one direct-Eulerian PPM sweep
// per pencil, written as a sequence of whole-pencil stages in the order the
// Enzo method paper describes them (Sec. "Hydrodynamics: The PPM method"):
//   1. pressure from the dual-energy selection rule (eta1),
//   2. CW84 limited slopes and interface values (CW84 Eqs. 1.6-1.8),
//   3. contact steepening of the density parabola (CW84 Eqs. 1.14-1.17),
//   4. shock flattening (CW84 appendix),
//   5. monotonicity constraint and parabola coefficients (CW84 Eq. 1.10 and
//      the paper's Eq. for q_{L}, Delta q, q_6),
//   6. characteristic tracing over the u-c, u, u+c domains (CW84 Eqs. 3.5-3.7),
//   7. two-shock Riemann solver and sampling at x/t = 0 (Sec. "Riemann
//      Solvers and Fallback"), or the HLLC flux when PPMO_HLLC is set,
//   8. fluxes and the conservative update of mass, momentum and total energy
//      (Eqs. mass_diff, momentum_diff, energy_diff, with the flux-difference
//      sign read as minus, i.e. the conservative upwind form) and of the
//      internal energy (Eq. gasenergy_diff), then the eta2 resync
//      (Eq. dualselect),
//   9. HLL fallback on faces of cells whose density or pressure went
//      non-positive (Sec. "Riemann Solvers and Fallback").
// The CFL reduction follows Sec. "Timestepping" (harmonic multi-D form).
//
// Every function is templated on the scalar type R only so that the same
// code can be instantiated with an operation-counting scalar (opcount.hpp);
// the public API instantiates R = double.  Build with -ffp-contract=off and no
// fast-math: the expressions below define the result bit for bit.

#include "ppm_oracle.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "opcount.hpp"

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// Parabola coefficients (CW84 Eqs. 1.5-1.6 on a uniform grid).
const double C16 = 1.0 / 6.0;
const double C23 = 2.0 / 3.0;
// Contact steepening constants (CW84 Eqs. 1.16-1.17 and 3.2).
// CW84's dissipation coefficient (the optional diffusive flux; CW84 is not
// available here, K = 0.1 is its published value as read).
const double DIFF_K = 0.1;
const double STEEP_EPS = 0.01;
const double STEEP_K0 = 0.1;
const double STEEP_ETA1 = 20.0;
const double STEEP_ETA2 = 0.05;
// Flattening constants (CW84 appendix).
const double FLAT_OMEGA1 = 0.75;
const double FLAT_OMEGA2 = 10.0;
const double FLAT_EPS = 0.33;

// Reconstructed and traced quantities.  The interface internal energy is not
// traced: it is the internal energy p/((g-1) rho) of the Riemann solution, the
// same state that gives the interface total energy.
enum { QR = 0, QU = 1, QV1 = 2, QV2 = 3, QP = 4, NQ = 5 };
enum { FR = 0, FU = 1, FV1 = 2, FV2 = 3, FE = 4, FEI = 5, FUB = 6, NF = 7 };

template <class R> R rmin(R a, R b) { return a < b ? a : b; }
template <class R> R rmax(R a, R b) { return a > b ? a : b; }
template <class R> R clamp01(R x) { return x < 0.0 ? R(0.0) : (x > 1.0 ? R(1.0) : x); }

using std::fabs;
using std::sqrt;

// The ratio test a/b > t of the paper's selection rules, taken as a > t*b
// when b > 0 (the case of every physical state) and as written otherwise.
template <class R> bool ratio_above(R a, R b, double t) {
  return b > 0.0 ? a > t * b : a / b > t;
}

// Average of the parabola over the part of the cell next to its right edge
// that a wave travelling right at Courant number y sweeps through in dt.
template <class R> R avg_right(R qr, R dq, R q6, R y) {
  return qr - 0.5 * y * (dq - (1.0 - C23 * y) * q6);
}
// Same next to the left edge, for a left-travelling wave.
template <class R> R avg_left(R ql, R dq, R q6, R y) {
  return ql + 0.5 * y * (dq + (1.0 - C23 * y) * q6);
}

template <class R> struct Work {
  std::vector<R> q[NQ], E, c, rhoE;
  std::vector<R> dm[NQ], face[NQ], ql[NQ], qr[NQ], dq[NQ], q6[NQ];
  std::vector<R> ftil;
  std::vector<R> stl[NQ], str[NQ];  // traced states at face j+1/2
  std::vector<R> F[NF];             // fluxes at face j+1/2
  std::vector<int> bad, hll;
  void resize(int n) {
    for (int k = 0; k < NQ; ++k) {
      q[k].assign(n, R(0.0)); dm[k].assign(n, R(0.0)); face[k].assign(n, R(0.0));
      ql[k].assign(n, R(0.0)); qr[k].assign(n, R(0.0)); dq[k].assign(n, R(0.0));
      q6[k].assign(n, R(0.0)); stl[k].assign(n, R(0.0)); str[k].assign(n, R(0.0));
    }
    for (int k = 0; k < NF; ++k) F[k].assign(n, R(0.0));
    E.assign(n, R(0.0)); c.assign(n, R(0.0)); rhoE.assign(n, R(0.0));
    ftil.assign(n, R(0.0));
    bad.assign(n, 0); hll.assign(n, 0);
  }
};

// ---------------------------------------------------------------------------
// Step 1: equation of state with the dual-energy selection (eta1 rule).
template <class R>
void eos(const ppmo_params &P, R rho, R u, R v1, R v2, R E, R e, R *p_out, R *c_out) {
  const double g = P.gamma;
  R ke = 0.5 * (u * u + v1 * v1 + v2 * v2);
  R eps = E - ke;
  if ((P.flags & PPMO_DUAL_ENERGY) && !ratio_above(eps, E, P.eta1)) eps = e;
  R p = (g - 1.0) * rho * eps;
  if (p < P.p_floor) p = R(P.p_floor);
  *p_out = p;
  *c_out = sqrt(g * p / rho);
}

// ---------------------------------------------------------------------------
// Step 7: two-shock Riemann solver.  Both waves are treated as shocks; the
// star pressure solves u*_R(p) = u*_L(p) by Newton's method, where
// u*_L = u_L - (p - p_L)/W_L, u*_R = u_R + (p - p_R)/W_R, W_s the Lagrangian
// shock speed C_s sqrt(1 + (g+1)/(2g) (p/p_s - 1)) and d u*_s/dp = -+1/Z_s,
// Z_s = 2 W_s^3 / (W_s^2 + C_s^2).
template <class R> struct RiemannOut {
  R ps, us, rho, u, p;
  int iters;
  bool left;
};

template <class R>
RiemannOut<R> two_shock(const ppmo_params &P, R rl, R ul, R pl, R rr, R ur, R pr) {
  const double g = P.gamma;
  const double G1 = (g + 1.0) / (2.0 * g);
  RiemannOut<R> o;
  R cl = sqrt(g * pl * rl);  // Lagrangian sound speeds
  R cr = sqrt(g * pr * rr);
  R ipl = 1.0 / pl, ipr = 1.0 / pr;
  // linearised (acoustic) first guess
  R ps = (cr * pl + cl * pr - cl * cr * (ur - ul)) / (cl + cr);
  if (ps < P.p_floor) ps = R(P.p_floor);
  // Iterate until the Newton correction falls below rtol; the star state is
  // that last iterate, with its shock speeds and contact velocities.
  int it = 0;
  bool capped = false;
  R wl, wr, iwl, iwr, usl, usr;
  for (;;) {
    wl = cl * sqrt(1.0 + G1 * (ps * ipl - 1.0));
    wr = cr * sqrt(1.0 + G1 * (ps * ipr - 1.0));
    iwl = 1.0 / wl;
    iwr = 1.0 / wr;
    usl = ul - (ps - pl) * iwl;
    usr = ur + (ps - pr) * iwr;
    if (capped || it == P.riemann_max_iter) break;
    // 1/Z_s = (W_s^2 + C_s^2) / (2 W_s^3)
    R izl = (wl * wl + cl * cl) * (0.5 * iwl * iwl * iwl);
    R izr = (wr * wr + cr * cr) * (0.5 * iwr * iwr * iwr);
    R pn = ps - (usr - usl) / (izl + izr);
    if (pn < P.p_floor) pn = R(P.p_floor);
    ++it;
    if (fabs(pn - ps) <= P.riemann_rtol * pn) break;  // ps is the answer
    ps = pn;
    if (it == P.riemann_max_iter) capped = true;  // evaluate at the last iterate
  }
  R us = 0.5 * (usl + usr);
  o.ps = ps; o.us = us; o.iters = it;
  // Sample the solution at x/t = 0.
  if (us >= 0.0) {
    o.left = true;
    R rs = 1.0 / (1.0 / rl - (ps - pl) * iwl * iwl);
    if (rs < P.rho_floor) rs = R(P.rho_floor);
    if (ps > pl) {  // left shock
      R s = ul - wl / rl;
      if (s >= 0.0) { o.rho = rl; o.u = ul; o.p = pl; }
      else { o.rho = rs; o.u = us; o.p = ps; }
    } else {        // left rarefaction, linear through the fan
      R head = ul - sqrt(g * pl / rl);
      R tail = us - sqrt(g * ps / rs);
      if (head >= 0.0) { o.rho = rl; o.u = ul; o.p = pl; }
      else if (tail <= 0.0) { o.rho = rs; o.u = us; o.p = ps; }
      else {
        R w = -head / (tail - head);
        o.rho = (1.0 - w) * rl + w * rs;
        o.u = (1.0 - w) * ul + w * us;
        o.p = (1.0 - w) * pl + w * ps;
      }
    }
  } else {
    o.left = false;
    R rs = 1.0 / (1.0 / rr - (ps - pr) * iwr * iwr);
    if (rs < P.rho_floor) rs = R(P.rho_floor);
    if (ps > pr) {  // right shock
      R s = ur + wr / rr;
      if (s <= 0.0) { o.rho = rr; o.u = ur; o.p = pr; }
      else { o.rho = rs; o.u = us; o.p = ps; }
    } else {        // right rarefaction
      R head = ur + sqrt(g * pr / rr);
      R tail = us + sqrt(g * ps / rs);
      if (head <= 0.0) { o.rho = rr; o.u = ur; o.p = pr; }
      else if (tail >= 0.0) { o.rho = rs; o.u = us; o.p = ps; }
      else {
        R w = head / (head - tail);
        o.rho = (1.0 - w) * rr + w * rs;
        o.u = (1.0 - w) * ur + w * us;
        o.p = (1.0 - w) * pr + w * ps;
      }
    }
  }
  return o;
}

// Fluxes from the sampled interface state (Eqs. mass_diff ... gasenergy_diff):
// F_rho = rho u, F_u = F_rho u + p, F_v = F_rho v, F_E = F_rho E + u p and
// F_e = F_rho e, with e = p/((g-1) rho) and E = e + |v|^2/2 of that state;
// transverse velocities come from the upwind side.  Slot FUB keeps the face
// velocity for the p div v term of the internal-energy equation.
template <class R>
void hllc_flux(const ppmo_params &P, const R *sl, const R *sr, R *F);

template <class R>
void godunov_flux(const ppmo_params &P, const R *sl, const R *sr, R *F) {
  if (P.flags & PPMO_HLLC) {
    hllc_flux<R>(P, sl, sr, F);
    return;
  }
  const double g = P.gamma;
  RiemannOut<R> o = two_shock<R>(P, sl[QR], sl[QU], sl[QP], sr[QR], sr[QU], sr[QP]);
  R v1 = o.left ? sl[QV1] : sr[QV1];
  R v2 = o.left ? sl[QV2] : sr[QV2];
  R fr = o.rho * o.u;
  F[FR] = fr;
  F[FU] = fr * o.u + o.p;
  F[FV1] = fr * v1;
  F[FV2] = fr * v2;
  R eb = o.p / ((g - 1.0) * o.rho);
  R Eb = eb + 0.5 * (o.u * o.u + v1 * v1 + v2 * v2);
  F[FE] = fr * Eb + o.u * o.p;
  F[FEI] = fr * eb;
  F[FUB] = o.u;
}

// HLL flux with Davis wave-speed estimates (fallback solver).
template <class R>
void hll_flux(const ppmo_params &P, const R *sl, const R *sr, R *F) {
  const double g = P.gamma;
  R rl = sl[QR], ul = sl[QU], pl = sl[QP];
  R rr = sr[QR], ur = sr[QU], pr = sr[QP];
  R cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
  R el = pl / ((g - 1.0) * rl), er = pr / ((g - 1.0) * rr);
  R El = el + 0.5 * (ul * ul + sl[QV1] * sl[QV1] + sl[QV2] * sl[QV2]);
  R Er = er + 0.5 * (ur * ur + sr[QV1] * sr[QV1] + sr[QV2] * sr[QV2]);
  R Ul[6] = {rl, rl * ul, rl * sl[QV1], rl * sl[QV2], rl * El, rl * el};
  R Ur[6] = {rr, rr * ur, rr * sr[QV1], rr * sr[QV2], rr * Er, rr * er};
  R Fl[6] = {rl * ul, rl * ul * ul + pl, rl * ul * sl[QV1], rl * ul * sl[QV2],
             ul * (rl * El + pl), rl * ul * el};
  R Fr[6] = {rr * ur, rr * ur * ur + pr, rr * ur * sr[QV1], rr * ur * sr[QV2],
             ur * (rr * Er + pr), rr * ur * er};
  R sL = rmin<R>(ul - cl, ur - cr);
  R sR = rmax<R>(ul + cl, ur + cr);
  if (sL >= 0.0) {
    for (int k = 0; k < 6; ++k) F[k] = Fl[k];
    F[FUB] = ul;
  } else if (sR <= 0.0) {
    for (int k = 0; k < 6; ++k) F[k] = Fr[k];
    F[FUB] = ur;
  } else {
    R id = 1.0 / (sR - sL);
    for (int k = 0; k < 6; ++k) F[k] = (sR * Fl[k] - sL * Fr[k] + sL * sR * (Ur[k] - Ul[k])) * id;
    // face velocity of the HLL intermediate state
    R um_r = (sR * Ur[0] - sL * Ul[0] - (Fr[0] - Fl[0])) * id;
    R um_m = (sR * Ur[1] - sL * Ul[1] - (Fr[1] - Fl[1])) * id;
    F[FUB] = um_m / um_r;
  }
}

// HLLC flux (Sec. "Riemann Solvers and Fallback": HLL with the contact wave
// restored), selected by PPMO_HLLC in place of the two-shock solver.  Outer
// wave speeds as in hll_flux (Davis estimates); the contact speed S* follows
// from the Rankine-Hugoniot conditions across the two outer waves with equal
// pressure and normal velocity on both sides of the contact; the state
// between an outer wave s_K and the contact is
//   rho*_K = rho_K (s_K - u_K) / (s_K - S*),  u* = S*,  v*_t = v_t,K,
//   E*_K = E_K + (S* - u_K) (S* + p_K / (rho_K (s_K - u_K))),
// the internal energy riding with the density (e*_K = e_K); the flux at
// x/t = 0 is that of the upwind side, F_K + s_K (U*_K - U_K) inside the fan.
// The face velocity slot carries S*.
template <class R>
void hllc_flux(const ppmo_params &P, const R *sl, const R *sr, R *F) {
  const double g = P.gamma;
  R rl = sl[QR], ul = sl[QU], pl = sl[QP];
  R rr = sr[QR], ur = sr[QU], pr = sr[QP];
  R cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
  R el = pl / ((g - 1.0) * rl), er = pr / ((g - 1.0) * rr);
  R El = el + 0.5 * (ul * ul + sl[QV1] * sl[QV1] + sl[QV2] * sl[QV2]);
  R Er = er + 0.5 * (ur * ur + sr[QV1] * sr[QV1] + sr[QV2] * sr[QV2]);
  R sL = rmin<R>(ul - cl, ur - cr);
  R sR = rmax<R>(ul + cl, ur + cr);
  // the side whose state (or star state) sits at x/t = 0
  R S = 0.0;
  bool left;
  if (sL >= 0.0) {
    left = true;
  } else if (sR <= 0.0) {
    left = false;
  } else {
    R ml = rl * (sL - ul), mr = rr * (sR - ur);
    S = (pr - pl + ml * ul - mr * ur) / (ml - mr);
    left = S >= 0.0;
  }
  R rK = left ? rl : rr, uK = left ? ul : ur, pK = left ? pl : pr;
  R v1K = left ? sl[QV1] : sr[QV1], v2K = left ? sl[QV2] : sr[QV2];
  R EK = left ? El : Er, eK = left ? el : er, sK = left ? sL : sR;
  R fr = rK * uK;
  R Fk[6] = {fr, fr * uK + pK, fr * v1K, fr * v2K, uK * (rK * EK + pK), fr * eK};
  if (sL >= 0.0 || sR <= 0.0) {
    for (int k = 0; k < 6; ++k) F[k] = Fk[k];
    F[FUB] = uK;
    return;
  }
  R mK = rK * (sK - uK);
  R rs = mK / (sK - S);
  R Us[6] = {rs, rs * S, rs * v1K, rs * v2K, rs * (EK + (S - uK) * (S + pK / mK)), rs * eK};
  R Uk[6] = {rK, rK * uK, rK * v1K, rK * v2K, rK * EK, rK * eK};
  for (int k = 0; k < 6; ++k) F[k] = Fk[k] + sK * (Us[k] - Uk[k]);
  F[FUB] = S;
}

template <class R> R minmod(R a, R b) {
  if (a * b < 0.0) return R(0.0);
  R m = fabs(a) < fabs(b) ? fabs(a) : fabs(b);
  return a < 0.0 ? -m : m;
}

template <class R> R corner_avg(const R (&nb)[3][3][3], int sx, int sy, int sz) {
  const int z0 = sz < 0 ? 0 : 1, y0 = sy < 0 ? 0 : 1, x0 = sx < 0 ? 0 : 1;
  R sum = 0.0;
  for (int z = z0; z <= z0 + 1; ++z)
    for (int y = y0; y <= y0 + 1; ++y)
      for (int x = x0; x <= x0 + 1; ++x) sum = sum + nb[z][y][x];
  return sum * 0.125;
}

template <class R> void second_order_a(const R (&nb)[3][3][3], int r, R *out) {
  const R q0 = nb[1][1][1];
  // diagonal n runs from corner -c_n to corner +c_n
  const int c[4][3] = {{1, 1, 1}, {-1, 1, 1}, {1, -1, 1}, {1, 1, -1}};
  R dq[4];
  for (int n = 0; n < 4; ++n) {
    R up = corner_avg<R>(nb, c[n][0], c[n][1], c[n][2]);
    R dn = corner_avg<R>(nb, -c[n][0], -c[n][1], -c[n][2]);
    dq[n] = minmod<R>(up - q0, q0 - dn);
  }
  const R sum = dq[1] + dq[2] + dq[3];
  bool adjust = false, chi[4] = {false, false, false, false};
  R target = 0.0;
  if (dq[0] != 0.0) {
    R s = sum / dq[0];
    if (s < 0.0 || s > 1.0) {
      adjust = true;
      target = dq[0] * (s < 0.0 ? R(0.0) : R(1.0));
      for (int n = 1; n < 4; ++n) {
        R ratio = dq[n] / dq[0];
        chi[n] = s < 0.0 ? ratio < 0.0 : ratio > 0.0;
      }
    }
  } else if (sum != 0.0) {  // the (+,+,+) change must vanish: scale those along the sum
    adjust = true;
    for (int n = 1; n < 4; ++n) chi[n] = sum > 0.0 ? dq[n] > 0.0 : dq[n] < 0.0;
  }
  if (adjust) {
    R sel = 0.0, rest = 0.0;
    for (int n = 1; n < 4; ++n) {
      if (chi[n]) sel = sel + dq[n];
      else rest = rest + dq[n];
    }
    R f = (target - rest) / sel;
    for (int n = 1; n < 4; ++n)
      if (chi[n]) dq[n] = f * dq[n];
  }
  const R fx = dq[2] + dq[3], fy = dq[1] + dq[3], fz = dq[1] + dq[2];
  for (int k = 0; k < r; ++k)
    for (int j = 0; j < r; ++j)
      for (int i = 0; i < r; ++i) {
        const R wx = (R(i) + (1.0 - r) * 0.5) / R(r);
        const R wy = (R(j) + (1.0 - r) * 0.5) / R(r);
        const R wz = (R(k) + (1.0 - r) * 0.5) / R(r);
        out[(k * r + j) * r + i] = q0 + wx * fx + wy * fy + wz * fz;
      }
}

int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Optional diffusive flux (Sec. "Hydrodynamics: The PPM method" refers to
// CW84's appendix for it), in its form along the sweep: where the flow
// converges across face j+1/2 (u_j > u_{j+1}, cell-centred normal
// velocities of the sweep input), every conserved quantity's face flux gains
// nu (Q_j - Q_{j+1}) with nu = K (u_j - u_{j+1}); nothing changes elsewhere.
// Q: rho, rho u, rho v1, rho v2, rho E, rho e; the face velocity of the
// p div v term is left alone.
template <class R>
void add_diffusion(const ppmo_params &P, const R *rho, const R *u, const R *v1, const R *v2,
                   const R *E, const R *e, int j, R *F) {
  if (!(P.flags & PPMO_DIFFUSION)) return;
  const R du = u[j] - u[j + 1];
  if (!(du > R(0.0))) return;
  const R nu = R(DIFF_K) * du;
  const R ql[6] = {rho[j], rho[j] * u[j], rho[j] * v1[j], rho[j] * v2[j], rho[j] * E[j],
                   rho[j] * e[j]};
  const R qr[6] = {rho[j + 1], rho[j + 1] * u[j + 1], rho[j + 1] * v1[j + 1],
                   rho[j + 1] * v2[j + 1], rho[j + 1] * E[j + 1], rho[j + 1] * e[j + 1]};
  for (int k = 0; k < 6; ++k) F[k] = F[k] + nu * (ql[k] - qr[k]);
}

// ---------------------------------------------------------------------------
// Step 8: conservative update of one active cell from its two face fluxes
// (Eqs. mass_diff, momentum_diff, energy_diff, gasenergy_diff; dtdx = dt /
// (a dx) in comoving coordinates), then the eta2 resync of e (Eq.
// dualselect).  With a gravity field, the time-centred source terms of Eqs.
// momentum_diff and energy_diff: momentum + (dt/2)(g/a)(rho^n + rho^{n+1}),
// total energy + (dt/2)(g/a)(rho^n u^n + rho^{n+1} u^{n+1}), with g the
// acceleration along the sweep at the cell centre (hg = 0.5 dt / a times it).
// Returns true when the new density or the eta1-selected new internal
// energy is not positive.
template <class R> struct CellIn { R rho, u, v1, v2, E, e, p, rhoEmax; };

template <class R>
bool update_cell(const ppmo_params &P, R dtdx, const CellIn<R> &c, const R *Fm, const R *Fp,
                 R *out, bool grav = false, R hg = R(0.0)) {
  const bool dual = (P.flags & PPMO_DUAL_ENERGY) != 0;
  R rn = c.rho - dtdx * (Fp[FR] - Fm[FR]);
  R mu = c.rho * c.u - dtdx * (Fp[FU] - Fm[FU]);
  R m1 = c.rho * c.v1 - dtdx * (Fp[FV1] - Fm[FV1]);
  R m2 = c.rho * c.v2 - dtdx * (Fp[FV2] - Fm[FV2]);
  R mE = c.rho * c.E - dtdx * (Fp[FE] - Fm[FE]);
  R me = c.rho * c.e - dtdx * (Fp[FEI] - Fm[FEI]) - dtdx * c.p * (Fp[FUB] - Fm[FUB]);
  if (grav) {
    mu = mu + hg * (c.rho + rn);
    mE = mE + hg * (c.rho * c.u + mu);
  }
  R ir = 1.0 / rn;
  R un = mu * ir, v1n = m1 * ir, v2n = m2 * ir, En = mE * ir, eraw = me * ir;
  R ke = 0.5 * (un * un + v1n * v1n + v2n * v2n);
  R epsE = En - ke;
  bool bad = !(rn > P.rho_floor);
  R sel = epsE;
  if (dual && !ratio_above(epsE, En, P.eta1)) sel = eraw;
  if (!(sel > 0.0)) bad = true;
  R en = eraw < P.e_floor ? R(P.e_floor) : eraw;
  if (dual && ratio_above(rn * epsE, c.rhoEmax, P.eta2)) en = epsE;
  out[0] = rn; out[1] = un; out[2] = v1n; out[3] = v2n; out[4] = En; out[5] = en;
  return bad;
}

// A cell still non-positive after the fallback: density raised to the floor
// (keeping the old velocity if so), pressure set to the floor.
template <class R>
void floor_cell(const ppmo_params &P, const CellIn<R> &c, R *out) {
  const double g = P.gamma;
  if (!(out[0] > P.rho_floor)) {
    out[0] = R(P.rho_floor);
    out[1] = c.u; out[2] = c.v1; out[3] = c.v2;
  }
  R eps = P.p_floor / ((g - 1.0) * out[0]);
  out[5] = eps;
  out[4] = eps + 0.5 * (out[1] * out[1] + out[2] * out[2] + out[3] * out[3]);
}

// ---------------------------------------------------------------------------
// One pencil sweep.  Cells 0..n-1 with gh ghost cells at each end: active
// cells a0 = gh .. a1 = n-gh-1, faces j+1/2 for j = a0-1..a1.  Reconstruction
// covers every cell whose stencil fits in the pencil.
template <class R>
void pencil_sweep(const ppmo_params &P, int n, int gh, R dt, R dx, R *rho, R *u, R *v1, R *v2,
                  R *Etot, R *eint, R *reg_lo, R *reg_hi, ppmo_counts *cnt, Work<R> &w,
                  const R *acc = nullptr) {
  const double g = P.gamma;
  const int a0 = gh, a1 = n - gh - 1;
  const R dtdx = dt / (P.a * dx);
  const R hgdt = 0.5 * dt / P.a;
  w.resize(n);
  R *a[NQ];
  for (int k = 0; k < NQ; ++k) a[k] = w.q[k].data();

  // 1. primitive state and pressure
  for (int j = 0; j < n; ++j) {
    a[QR][j] = rho[j]; a[QU][j] = u[j]; a[QV1][j] = v1[j]; a[QV2][j] = v2[j];
    w.E[j] = Etot[j];
    eos<R>(P, rho[j], u[j], v1[j], v2[j], Etot[j], eint[j], &a[QP][j], &w.c[j]);
    w.rhoE[j] = rho[j] * Etot[j];
  }

  // 2. limited slopes (j = 1..n-2) and interface values q_{j+1/2} (j = 1..n-3)
  for (int k = 0; k < NQ; ++k) {
    R *q = a[k], *dm = w.dm[k].data();
    for (int j = 1; j <= n - 2; ++j) {
      R dl = q[j] - q[j - 1], dr = q[j + 1] - q[j];
      R dc = 0.5 * (q[j + 1] - q[j - 1]);
      R m = 0.0;
      if (dl * dr > 0.0) {
        m = fabs(dc);
        if (2.0 * fabs(dl) < m) m = 2.0 * fabs(dl);
        if (2.0 * fabs(dr) < m) m = 2.0 * fabs(dr);
        if (dc < 0.0) m = -m;
      }
      dm[j] = m;
    }
    for (int j = 1; j <= n - 3; ++j)
      w.face[k][j] = 0.5 * (q[j] + q[j + 1]) - C16 * (dm[j + 1] - dm[j]);
    for (int j = 2; j <= n - 3; ++j) {
      w.ql[k][j] = w.face[k][j - 1];
      w.qr[k][j] = w.face[k][j];
    }
  }

  // 3. contact steepening of the density parabola (cells 2..n-3)
  if (P.flags & PPMO_STEEPEN) {
    R *r = a[QR], *p = a[QP], *dm = w.dm[QR].data();
    for (int j = 2; j <= n - 3; ++j) {
      R d2m = r[j] - 2.0 * r[j - 1] + r[j - 2];  // second difference at j-1
      R d2p = r[j + 2] - 2.0 * r[j + 1] + r[j];  // second difference at j+1
      R drho = r[j + 1] - r[j - 1];
      R eta = 0.0;
      if (d2p * d2m < 0.0 &&
          fabs(drho) - STEEP_EPS * rmin<R>(fabs(r[j + 1]), fabs(r[j - 1])) > 0.0 &&
          g * STEEP_K0 * fabs(drho) * rmin<R>(p[j + 1], p[j - 1]) >=
              fabs(p[j + 1] - p[j - 1]) * rmin<R>(r[j + 1], r[j - 1])) {
        R etat = -(d2p - d2m) / (6.0 * drho);
        eta = clamp01<R>(STEEP_ETA1 * (etat - STEEP_ETA2));
      }
      w.ql[QR][j] = w.ql[QR][j] * (1.0 - eta) + (r[j - 1] + 0.5 * dm[j - 1]) * eta;
      w.qr[QR][j] = w.qr[QR][j] * (1.0 - eta) + (r[j + 1] - 0.5 * dm[j + 1]) * eta;
    }
  }

  // 4. shock flattening.  ftil is zero where its stencil (j-2..j+2) would
  //    leave the pencil, i.e. outside cells 2..n-3.
  if (P.flags & PPMO_FLATTEN) {
    R *p = a[QP], *uu = a[QU];
    for (int j = 2; j <= n - 3; ++j) {
      R dp = p[j + 1] - p[j - 1];
      R f = 0.0;
      if (fabs(dp) > FLAT_EPS * rmin<R>(p[j + 1], p[j - 1]) && uu[j - 1] - uu[j + 1] > 0.0) {
        R den = p[j + 2] - p[j - 2];
        if (den == 0.0) f = 1.0;
        else f = clamp01<R>(FLAT_OMEGA2 * (dp / den - FLAT_OMEGA1));
      }
      w.ftil[j] = f;
    }
    for (int j = 2; j <= n - 3; ++j) {
      R fn = (p[j + 1] - p[j - 1] > 0.0) ? w.ftil[j - 1] : w.ftil[j + 1];
      R f = rmax<R>(w.ftil[j], fn);
      for (int k = 0; k < NQ; ++k) {
        w.ql[k][j] = f * a[k][j] + (1.0 - f) * w.ql[k][j];
        w.qr[k][j] = f * a[k][j] + (1.0 - f) * w.qr[k][j];
      }
    }
  }

  // 5. monotonicity (CW84 Eq. 1.10) and Delta q, q_6
  for (int k = 0; k < NQ; ++k) {
    for (int j = 2; j <= n - 3; ++j) {
      R q = a[k][j], l = w.ql[k][j], r = w.qr[k][j];
      if ((r - q) * (q - l) <= 0.0) {
        l = q;
        r = q;
      } else {
        R d = r - l;
        R s = d * (q - 0.5 * (l + r));
        R d2 = d * d * C16;
        if (s > d2) l = 3.0 * q - 2.0 * r;
        else if (-d2 > s) r = 3.0 * q - 2.0 * l;
      }
      w.ql[k][j] = l;
      w.qr[k][j] = r;
      w.dq[k][j] = r - l;
      w.q6[k][j] = 6.0 * (q - 0.5 * (l + r));
    }
  }

  // 6. characteristic tracing (CW84 Eqs. 3.5-3.7).  The reference state is
  //    the average over the domain of the fastest wave reaching the face; the
  //    beta corrections project the other waves' averages onto the linearised
  //    characteristic fields p +- C u and 1/rho + p/C^2.
  for (int j = a0 - 1; j <= a1; ++j) {
    // left state at face j+1/2, from cell j (waves moving right)
    {
      const int m = j;
      R uc = a[QU][m], cc = w.c[m];
      R ym = clamp01<R>((uc - cc) * dtdx);
      R y0 = clamp01<R>(uc * dtdx);
      R yp = clamp01<R>((uc + cc) * dtdx);
      R rt = avg_right<R>(w.qr[QR][m], w.dq[QR][m], w.q6[QR][m], yp);
      R ut = avg_right<R>(w.qr[QU][m], w.dq[QU][m], w.q6[QU][m], yp);
      R pt = avg_right<R>(w.qr[QP][m], w.dq[QP][m], w.q6[QP][m], yp);
      R C = sqrt(g * pt * rt);
      R iC = 1.0 / C;
      R bp = 0.0, bm = 0.0, b0 = 0.0;
      if (uc + cc > 0.0) {
        R up = avg_right<R>(w.qr[QU][m], w.dq[QU][m], w.q6[QU][m], yp);
        R pp = avg_right<R>(w.qr[QP][m], w.dq[QP][m], w.q6[QP][m], yp);
        bp = -0.5 * iC * ((ut - up) + (pt - pp) * iC);
      }
      if (uc - cc > 0.0) {
        R um = avg_right<R>(w.qr[QU][m], w.dq[QU][m], w.q6[QU][m], ym);
        R pm = avg_right<R>(w.qr[QP][m], w.dq[QP][m], w.q6[QP][m], ym);
        bm = 0.5 * iC * ((ut - um) - (pt - pm) * iC);
      }
      if (uc > 0.0) {
        R r0 = avg_right<R>(w.qr[QR][m], w.dq[QR][m], w.q6[QR][m], y0);
        R p0 = avg_right<R>(w.qr[QP][m], w.dq[QP][m], w.q6[QP][m], y0);
        b0 = (pt - p0) * iC * iC + 1.0 / rt - 1.0 / r0;
      }
      R ps = pt + C * C * (bp + bm);
      R us = ut + C * (bp - bm);
      R tau = 1.0 / rt - (bp + bm + b0);
      R rs = tau > 0.0 ? 1.0 / tau : rt;
      w.stl[QR][j] = rmax<R>(rs, R(P.rho_floor));
      w.stl[QU][j] = us;
      w.stl[QP][j] = rmax<R>(ps, R(P.p_floor));
      w.stl[QV1][j] = avg_right<R>(w.qr[QV1][m], w.dq[QV1][m], w.q6[QV1][m], y0);
      w.stl[QV2][j] = avg_right<R>(w.qr[QV2][m], w.dq[QV2][m], w.q6[QV2][m], y0);
    }
    // right state at face j+1/2, from cell j+1 (waves moving left)
    {
      const int m = j + 1;
      R uc = a[QU][m], cc = w.c[m];
      R ym = clamp01<R>(-(uc - cc) * dtdx);
      R y0 = clamp01<R>(-uc * dtdx);
      R yp = clamp01<R>(-(uc + cc) * dtdx);
      R rt = avg_left<R>(w.ql[QR][m], w.dq[QR][m], w.q6[QR][m], ym);
      R ut = avg_left<R>(w.ql[QU][m], w.dq[QU][m], w.q6[QU][m], ym);
      R pt = avg_left<R>(w.ql[QP][m], w.dq[QP][m], w.q6[QP][m], ym);
      R C = sqrt(g * pt * rt);
      R iC = 1.0 / C;
      R bp = 0.0, bm = 0.0, b0 = 0.0;
      if (uc - cc < 0.0) {
        R um = avg_left<R>(w.ql[QU][m], w.dq[QU][m], w.q6[QU][m], ym);
        R pm = avg_left<R>(w.ql[QP][m], w.dq[QP][m], w.q6[QP][m], ym);
        bm = 0.5 * iC * ((ut - um) - (pt - pm) * iC);
      }
      if (uc + cc < 0.0) {
        R up = avg_left<R>(w.ql[QU][m], w.dq[QU][m], w.q6[QU][m], yp);
        R pp = avg_left<R>(w.ql[QP][m], w.dq[QP][m], w.q6[QP][m], yp);
        bp = -0.5 * iC * ((ut - up) + (pt - pp) * iC);
      }
      if (uc < 0.0) {
        R r0 = avg_left<R>(w.ql[QR][m], w.dq[QR][m], w.q6[QR][m], y0);
        R p0 = avg_left<R>(w.ql[QP][m], w.dq[QP][m], w.q6[QP][m], y0);
        b0 = (pt - p0) * iC * iC + 1.0 / rt - 1.0 / r0;
      }
      R ps = pt + C * C * (bp + bm);
      R us = ut + C * (bp - bm);
      R tau = 1.0 / rt - (bp + bm + b0);
      R rs = tau > 0.0 ? 1.0 / tau : rt;
      w.str[QR][j] = rmax<R>(rs, R(P.rho_floor));
      w.str[QU][j] = us;
      w.str[QP][j] = rmax<R>(ps, R(P.p_floor));
      w.str[QV1][j] = avg_left<R>(w.ql[QV1][m], w.dq[QV1][m], w.q6[QV1][m], y0);
      w.str[QV2][j] = avg_left<R>(w.ql[QV2][m], w.dq[QV2][m], w.q6[QV2][m], y0);
    }
  }

  // 7. Riemann problems and fluxes at faces j+1/2, j = a0-1..a1 (with the
  //    optional diffusive flux)
  for (int j = a0 - 1; j <= a1; ++j) {
    R sl[NQ], sr[NQ], F[NF];
    for (int k = 0; k < NQ; ++k) { sl[k] = w.stl[k][j]; sr[k] = w.str[k][j]; }
    godunov_flux<R>(P, sl, sr, F);
    add_diffusion<R>(P, rho, u, v1, v2, Etot, eint, j, F);
    for (int k = 0; k < NF; ++k) w.F[k][j] = F[k];
  }

  // 8. provisional update of the active cells
  std::vector<R> out((size_t)n * 6, R(0.0));
  auto cell_in = [&](int j) {
    CellIn<R> c;
    c.rho = rho[j]; c.u = u[j]; c.v1 = v1[j]; c.v2 = v2[j]; c.E = Etot[j]; c.e = eint[j];
    c.p = a[QP][j];
    c.rhoEmax = rmax<R>(rmax<R>(w.rhoE[j - 1], w.rhoE[j]), w.rhoE[j + 1]);
    return c;
  };
  auto do_update = [&](int j) {
    R Fm[NF], Fp[NF];
    for (int k = 0; k < NF; ++k) { Fm[k] = w.F[k][j - 1]; Fp[k] = w.F[k][j]; }
    return update_cell<R>(P, dtdx, cell_in(j), Fm, Fp, &out[(size_t)j * 6], acc != nullptr,
                          acc ? hgdt * acc[j] : R(0.0));
  };
  for (int j = 0; j < n; ++j) w.bad[j] = 0;
  for (int j = a0; j <= a1; ++j) w.bad[j] = do_update(j) ? 1 : 0;

  // 9. fallback: re-solve every face of a non-positive cell with HLL and
  //    redo the update of every cell touching such a face (one pass).
  if (P.flags & PPMO_FALLBACK_HLL) {
    bool any = false;
    for (int j = a0 - 1; j <= a1; ++j) {
      w.hll[j] = (w.bad[j] || w.bad[j + 1]) ? 1 : 0;
      if (w.hll[j]) {
        any = true;
        R sl[NQ], sr[NQ], F[NF];
        for (int k = 0; k < NQ; ++k) { sl[k] = w.stl[k][j]; sr[k] = w.str[k][j]; }
        hll_flux<R>(P, sl, sr, F);
        add_diffusion<R>(P, rho, u, v1, v2, Etot, eint, j, F);
        for (int k = 0; k < NF; ++k) w.F[k][j] = F[k];
        if (cnt) cnt->fallback_faces++;
      }
    }
    if (any)
      for (int j = a0; j <= a1; ++j)
        if (w.hll[j - 1] || w.hll[j]) w.bad[j] = do_update(j) ? 1 : 0;
  }
  for (int j = a0; j <= a1; ++j)
    if (w.bad[j]) {
      floor_cell<R>(P, cell_in(j), &out[(size_t)j * 6]);
      if (cnt) cnt->floored_cells++;
    }

  // write back the active cells
  for (int j = a0; j <= a1; ++j) {
    const R *o = &out[(size_t)j * 6];
    rho[j] = o[0]; u[j] = o[1]; v1[j] = o[2]; v2[j] = o[3]; Etot[j] = o[4]; eint[j] = o[5];
  }
  // boundary flux registers: dt * F at the first and last active faces
  if (reg_lo)
    for (int k = 0; k < 6; ++k) reg_lo[k] = dt * w.F[k][a0 - 1];
  if (reg_hi)
    for (int k = 0; k < 6; ++k) reg_hi[k] = dt * w.F[k][a1];
}

// ---------------------------------------------------------------------------
// Grid-level drivers.

bool valid_grid(const ppmo_grid *g) {
  return g && g->nx >= 1 && g->ny >= 1 && g->nz >= 1 && g->ghost >= 3 && g->ghost <= 6 &&
         g->dx > 0 &&
         g->dy > 0 && g->dz > 0 && g->rho && g->vx && g->vy && g->vz && g->etot && g->eint &&
         ((g->gx && g->gy && g->gz) || (!g->gx && !g->gy && !g->gz));
}
bool valid_params(const ppmo_params *p) {
  return p && p->gamma > 1.0 && p->cfl > 0.0 && p->cfl <= 1.0 && p->riemann_max_iter >= 1 &&
         p->riemann_rtol > 0.0 && p->rho_floor > 0.0 && p->p_floor > 0.0 && p->e_floor > 0.0 &&
         p->a > 0.0 && std::isfinite(p->a) && std::isfinite(p->adot);
}

// Offset of face f's block in a grid's flux register.
int64_t reg_face_offset(int nx, int ny, int nz, int face) {
  int64_t area[3] = {(int64_t)ny * nz, (int64_t)nx * nz, (int64_t)nx * ny};
  int64_t off = 0;
  for (int f = 0; f < face; ++f) off += 6 * area[f / 2];
  return off;
}

// Boxes of active cells (a finer patch's footprint) whose boundary fluxes a
// step records: the faces lo[a]-1/2 and hi[a]-1/2 of each axis a, for the
// pencils along a whose transverse cells lie in the box, as dt * F in the
// layout of a flux register of a grid with the box's dimensions.
struct Capture {
  const ppmo_box *boxes = nullptr;
  int nboxes = 0;
  double *out = nullptr;
};

int64_t box_dim(const ppmo_box &b, int a) { return (int64_t)b.hi[a] - b.lo[a]; }

template <class R>
int sweep_impl(ppmo_grid *G, const ppmo_params *P, double dt, int axis, int active_mask,
               ppmo_counts *counts, const Capture &cap = Capture()) {
  const int g = G->ghost;
  const int N[3] = {G->nx, G->ny, G->nz};
  const int64_t n[3] = {N[0] + 2 * g, N[1] + 2 * g, N[2] + 2 * g};
  const int64_t stride[3] = {1, n[0], n[0] * n[1]};
  const double dxs[3] = {G->dx, G->dy, G->dz};
  double *vel[3] = {G->vx, G->vy, G->vz};
  const int t1 = axis == 0 ? 1 : 0, t2 = axis == 2 ? 1 : 2;
  const int lo1 = (active_mask >> t1) & 1 ? g : 0, hi1 = (active_mask >> t1) & 1 ? g + N[t1] : n[t1];
  const int lo2 = (active_mask >> t2) & 1 ? g : 0, hi2 = (active_mask >> t2) & 1 ? g + N[t2] : n[t2];
  const int len = (int)n[axis];
  const int64_t np = (int64_t)(hi1 - lo1) * (hi2 - lo2);
  int64_t fb = 0, fl = 0;
  // register blocks (only for pencils whose transverse indices are active)
  double *reg_lo_base = nullptr, *reg_hi_base = nullptr;
  int64_t reg_field_stride = 0;
  if (G->flux_reg) {
    reg_lo_base = G->flux_reg + reg_face_offset(N[0], N[1], N[2], 2 * axis);
    reg_hi_base = G->flux_reg + reg_face_offset(N[0], N[1], N[2], 2 * axis + 1);
    reg_field_stride = (int64_t)N[t1] * N[t2];
  }
  // lab index of each pencil-local flux slot rho,u,v1,v2,E,e
  const int lab_of[6] = {0, 1 + axis, 1 + t1, 1 + t2, 4, 5};

#pragma omp parallel reduction(+ : fb, fl)
  {
    Work<R> w;
    std::vector<R> r(len), uu(len), a1(len), a2(len), E(len), e(len), ga(len);
    std::vector<R> rl(6), rh(6);
    const double *gfield = axis == 0 ? G->gx : (axis == 1 ? G->gy : G->gz);
    ppmo_counts c = {0, 0};
#pragma omp for schedule(static)
    for (int64_t ip = 0; ip < np; ++ip) {
      const int i1 = lo1 + (int)(ip % (hi1 - lo1));
      const int i2 = lo2 + (int)(ip / (hi1 - lo1));
      const int64_t base = i1 * stride[t1] + i2 * stride[t2];
      for (int k = 0; k < len; ++k) {
        const int64_t o = base + k * stride[axis];
        r[k] = G->rho[o]; uu[k] = vel[axis][o]; a1[k] = vel[t1][o]; a2[k] = vel[t2][o];
        E[k] = G->etot[o]; e[k] = G->eint[o];
        if (gfield) ga[k] = gfield[o];
      }
      const bool reg = G->flux_reg && i1 >= g && i1 < g + N[t1] && i2 >= g && i2 < g + N[t2];
      pencil_sweep<R>(*P, len, g, R(dt), R(dxs[axis]), r.data(), uu.data(), a1.data(), a2.data(),
                      E.data(), e.data(), reg ? rl.data() : nullptr, reg ? rh.data() : nullptr,
                      &c, w, gfield ? ga.data() : nullptr);
      for (int k = g; k < g + N[axis]; ++k) {
        const int64_t o = base + k * stride[axis];
        G->rho[o] = opc_val(r[k]); vel[axis][o] = opc_val(uu[k]);
        vel[t1][o] = opc_val(a1[k]); vel[t2][o] = opc_val(a2[k]);
        G->etot[o] = opc_val(E[k]); G->eint[o] = opc_val(e[k]);
      }
      if (reg) {
        const int64_t ro = (int64_t)(i2 - g) * N[t1] + (i1 - g);
        for (int k = 0; k < 6; ++k) {
          reg_lo_base[lab_of[k] * reg_field_stride + ro] = opc_val(rl[k]);
          reg_hi_base[lab_of[k] * reg_field_stride + ro] = opc_val(rh[k]);
        }
      }
      // fluxes through the faces of capture boxes crossed by this pencil
      // (w.F holds the final fluxes of faces a0-1 .. a1; face j is j+1/2)
      int64_t boff = 0;
      for (int b = 0; b < cap.nboxes; ++b) {
        const ppmo_box &B = cap.boxes[b];
        const int64_t bd[3] = {box_dim(B, 0), box_dim(B, 1), box_dim(B, 2)};
        const int c1 = i1 - g - B.lo[t1], c2 = i2 - g - B.lo[t2];
        if (c1 >= 0 && c1 < bd[t1] && c2 >= 0 && c2 < bd[t2]) {
          const int64_t fs = bd[t1] * bd[t2], ro = (int64_t)c2 * bd[t1] + c1;
          const int jf[2] = {g + B.lo[axis] - 1, g + B.hi[axis] - 1};
          for (int side = 0; side < 2; ++side) {
            double *dst = cap.out + boff + reg_face_offset((int)bd[0], (int)bd[1], (int)bd[2],
                                                           2 * axis + side);
            for (int k = 0; k < 6; ++k)
              dst[lab_of[k] * fs + ro] = opc_val(R(dt) * w.F[k][jf[side]]);
          }
        }
        boff += reg_face_offset((int)bd[0], (int)bd[1], (int)bd[2], 6);
      }
    }
    fb += c.fallback_faces;
    fl += c.floored_cells;
  }
  if (counts) {
    counts->fallback_faces += fb;
    counts->floored_cells += fl;
  }
  return 0;
}

const int kOrders[6][3] = {{0, 1, 2}, {2, 1, 0}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}};

template <class R>
int step_impl(ppmo_grid *G, const ppmo_params *P, double dt, int order, ppmo_counts *counts,
              const Capture &cap = Capture()) {
  int mask = 0;
  for (int s = 0; s < 3; ++s) {
    const int axis = kOrders[order][s];
    mask |= 1 << axis;  // axes swept so far (including this one) are restricted
    sweep_impl<R>(G, P, dt, axis, mask & ~(1 << axis), counts, cap);
  }
  return 0;
}

bool box_inside(const ppmo_grid *G, const ppmo_box &b, int margin) {
  const int N[3] = {G->nx, G->ny, G->nz};
  for (int a = 0; a < 3; ++a)
    if (b.lo[a] < margin || b.hi[a] > N[a] - margin || b.hi[a] <= b.lo[a]) return false;
  return true;
}

bool in_box(const ppmo_box &b, int x, int y, int z) {
  return x >= b.lo[0] && x < b.hi[0] && y >= b.lo[1] && y < b.hi[1] && z >= b.lo[2] &&
         z < b.hi[2];
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

int64_t ppmo_flux_reg_size(int32_t nx, int32_t ny, int32_t nz) {
  return reg_face_offset(nx, ny, nz, 6);
}

int ppmo_sweep(ppmo_grid *g, const ppmo_params *p, double dt, int32_t axis,
               int32_t active_mask, ppmo_counts *counts) {
  if (!valid_grid(g) || !valid_params(p) || axis < 0 || axis > 2 || !(dt > 0)) return -1;
  return sweep_impl<double>(g, p, dt, axis, active_mask, counts);
}

int ppmo_step(ppmo_grid *g, const ppmo_params *p, double dt, int32_t order,
              ppmo_counts *counts) {
  if (!valid_grid(g) || !valid_params(p) || order < 0 || order > 5 || !(dt > 0)) return -1;
  return step_impl<double>(g, p, dt, order, counts);
}

int ppmo_step_capture(ppmo_grid *g, const ppmo_params *p, double dt, int32_t order,
                      ppmo_counts *counts, const ppmo_box *boxes, int32_t nboxes, double *out) {
  if (!valid_grid(g) || !valid_params(p) || order < 0 || order > 5 || !(dt > 0) ||
      nboxes < 0 || (nboxes > 0 && (!boxes || !out)))
    return -1;
  for (int b = 0; b < nboxes; ++b)
    if (!box_inside(g, boxes[b], 0)) return -1;
  Capture cap;
  cap.boxes = boxes;
  cap.nboxes = nboxes;
  cap.out = out;
  return step_impl<double>(g, p, dt, order, counts, cap);
}

int ppmo_flux_correct(ppmo_grid *C, const ppmo_params *P, const ppmo_box *boxes,
                      int32_t nboxes, const double *caps, const double *fine_sums, int32_t r) {
  if (!valid_grid(C) || !valid_params(P) || r < 2 || nboxes < 0 ||
      (nboxes > 0 && (!boxes || !caps || !fine_sums)))
    return -1;
  for (int b = 0; b < nboxes; ++b)
    if (!box_inside(C, boxes[b], 1)) return -1;
  const int g = C->ghost;
  const int N[3] = {C->nx, C->ny, C->nz};
  const int64_t n[3] = {N[0] + 2 * g, N[1] + 2 * g, N[2] + 2 * g};
  const double dxs[3] = {C->dx, C->dy, C->dz};
  // accumulated change of the conserved quantities rho, rho v, rho E, rho e
  // of each coarse cell, contributions added in box, face, cell order
  std::vector<double> delta((size_t)n[0] * n[1] * n[2] * 6, 0.0);
  std::vector<char> touched((size_t)n[0] * n[1] * n[2], 0);
  int64_t coff = 0, foff = 0;
  for (int b = 0; b < nboxes; ++b) {
    const ppmo_box &B = boxes[b];
    const int bd[3] = {B.hi[0] - B.lo[0], B.hi[1] - B.lo[1], B.hi[2] - B.lo[2]};
    const int fd[3] = {bd[0] * r, bd[1] * r, bd[2] * r};  // the fine patch's active dims
    for (int face = 0; face < 6; ++face) {
      const int a = face / 2, side = face % 2;
      const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
      const int64_t cfs = (int64_t)bd[t1] * bd[t2], ffs = (int64_t)fd[t1] * fd[t2];
      const double *cface = caps + coff + reg_face_offset(bd[0], bd[1], bd[2], face);
      const double *fface = fine_sums + foff + reg_face_offset(fd[0], fd[1], fd[2], face);
      for (int c2 = 0; c2 < bd[t2]; ++c2)
        for (int c1 = 0; c1 < bd[t1]; ++c1) {
          // the coarse cell just outside this face
          int c[3];
          c[a] = side == 0 ? B.lo[a] - 1 : B.hi[a];
          c[t1] = B.lo[t1] + c1;
          c[t2] = B.lo[t2] + c2;
          bool covered = false;
          for (int o = 0; o < nboxes && !covered; ++o) covered = in_box(boxes[o], c[0], c[1], c[2]);
          if (covered) continue;
          const int64_t cell = ((int64_t)(c[2] + g) * n[1] + (c[1] + g)) * n[0] + (c[0] + g);
          touched[cell] = 1;
          for (int k = 0; k < 6; ++k) {
            // area average of the r x r fine faces that make up the coarse face
            double sum = 0.0;
            for (int jj = 0; jj < r; ++jj)
              for (int ii = 0; ii < r; ++ii)
                sum += fface[k * ffs + (int64_t)(c2 * r + jj) * fd[t1] + (c1 * r + ii)];
            const double fine = sum / (double)(r * r);
            const double coarse = cface[k * cfs + (int64_t)c2 * bd[t1] + c1];
            // the outside cell's update used the coarse flux through this face
            // (its +a face on the low side, its -a face on the high side)
            const double d = side == 0 ? coarse - fine : fine - coarse;
            delta[(size_t)cell * 6 + k] += d / (P->a * dxs[a]);
          }
        }
    }
    coff += reg_face_offset(bd[0], bd[1], bd[2], 6);
    foff += reg_face_offset(fd[0], fd[1], fd[2], 6);
  }
  for (size_t cell = 0; cell < touched.size(); ++cell) {
    if (!touched[cell]) continue;
    const double *dq = &delta[cell * 6];
    const double rho = C->rho[cell];
    const double rn = rho + dq[0];
    const double mx = rho * C->vx[cell] + dq[1];
    const double my = rho * C->vy[cell] + dq[2];
    const double mz = rho * C->vz[cell] + dq[3];
    const double mE = rho * C->etot[cell] + dq[4];
    const double me = rho * C->eint[cell] + dq[5];
    C->rho[cell] = rn;
    C->vx[cell] = mx / rn;
    C->vy[cell] = my / rn;
    C->vz[cell] = mz / rn;
    C->etot[cell] = mE / rn;
    C->eint[cell] = me / rn;
  }
  return 0;
}

int ppmo_project(ppmo_grid *C, const ppmo_box *box, const ppmo_grid *F, int32_t r) {
  if (!valid_grid(C) || !valid_grid(F) || !box || r < 2 || !box_inside(C, *box, 0)) return -1;
  const ppmo_box &B = *box;
  if (F->nx != r * (B.hi[0] - B.lo[0]) || F->ny != r * (B.hi[1] - B.lo[1]) ||
      F->nz != r * (B.hi[2] - B.lo[2]))
    return -1;
  const int gc = C->ghost, gf = F->ghost;
  const int64_t nc[3] = {C->nx + 2 * gc, C->ny + 2 * gc, C->nz + 2 * gc};
  const int64_t nf[3] = {F->nx + 2 * gf, F->ny + 2 * gf, F->nz + 2 * gf};
  const double vol = (double)(r * r * r);
  for (int z = B.lo[2]; z < B.hi[2]; ++z)
    for (int y = B.lo[1]; y < B.hi[1]; ++y)
      for (int x = B.lo[0]; x < B.hi[0]; ++x) {
        // volume average of the conserved quantities of the r^3 fine cells
        double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int kk = 0; kk < r; ++kk)
          for (int jj = 0; jj < r; ++jj)
            for (int ii = 0; ii < r; ++ii) {
              const int64_t fx = gf + (int64_t)(x - B.lo[0]) * r + ii;
              const int64_t fy = gf + (int64_t)(y - B.lo[1]) * r + jj;
              const int64_t fz = gf + (int64_t)(z - B.lo[2]) * r + kk;
              const int64_t o = (fz * nf[1] + fy) * nf[0] + fx;
              const double rho = F->rho[o];
              s[0] += rho;
              s[1] += rho * F->vx[o];
              s[2] += rho * F->vy[o];
              s[3] += rho * F->vz[o];
              s[4] += rho * F->etot[o];
              s[5] += rho * F->eint[o];
            }
        const int64_t o = ((int64_t)(z + gc) * nc[1] + (y + gc)) * nc[0] + (x + gc);
        const double rho = s[0] / vol;
        C->rho[o] = rho;
        C->vx[o] = (s[1] / vol) / rho;
        C->vy[o] = (s[2] / vol) / rho;
        C->vz[o] = (s[3] / vol) / rho;
        C->etot[o] = (s[4] / vol) / rho;
        C->eint[o] = (s[5] / vol) / rho;
      }
  return 0;
}

int ppmo_pencil(const ppmo_params *p, int32_t n, int32_t ghost, double dt, double dx,
                double *rho, double *u, double *v1, double *v2, double *etot, double *eint,
                double *reg_lo, double *reg_hi, ppmo_counts *counts) {
  if (!valid_params(p) || ghost < 3 || ghost > 6 || n < 2 * ghost + 1 || !(dt > 0) ||
      !(dx > 0))
    return -1;
  Work<double> w;
  ppmo_counts c = {0, 0};
  pencil_sweep<double>(*p, n, ghost, dt, dx, rho, u, v1, v2, etot, eint, reg_lo, reg_hi, &c,
                       w);
  if (counts) {
    counts->fallback_faces += c.fallback_faces;
    counts->floored_cells += c.floored_cells;
  }
  return 0;
}

double ppmo_cfl_signal_max(const ppmo_grid *G, const ppmo_params *P) {
  if (!valid_grid(G) || !valid_params(P)) return -1.0;
  const int g = G->ghost;
  const int64_t nx = G->nx + 2 * g, ny = G->ny + 2 * g;
  double smax = 0.0;
  for (int k = g; k < g + G->nz; ++k)
    for (int j = g; j < g + G->ny; ++j)
      for (int i = g; i < g + G->nx; ++i) {
        const int64_t o = (k * ny + j) * nx + i;
        double p, c;
        eos<double>(*P, G->rho[o], G->vx[o], G->vy[o], G->vz[o], G->etot[o], G->eint[o], &p,
                    &c);
        double s = (c + fabs(G->vx[o])) / G->dx + (c + fabs(G->vy[o])) / G->dy +
                   (c + fabs(G->vz[o])) / G->dz;
        if (s > smax) smax = s;
      }
  return smax;
}

double ppmo_cfl_dt(const ppmo_grid *G, const ppmo_params *P) {
  double s = ppmo_cfl_signal_max(G, P);
  if (!(s > 0)) return -1.0;
  return (P->cfl * P->a) / s;  // Eq. dthydro: kappa a dx / (c_s + |v|)
}

int ppmo_expansion(ppmo_grid *G, const ppmo_params *P, double dt) {
  if (!valid_grid(G) || !valid_params(P) || !(dt >= 0)) return -1;
  const int g = G->ghost;
  const int N[3] = {G->nx, G->ny, G->nz};
  const int64_t n[3] = {N[0] + 2 * g, N[1] + 2 * g, N[2] + 2 * g};
  const double H = P->adot / P->a;
  const double xv = 0.5 * H * dt, xE = H * dt, xe = 1.5 * (P->gamma - 1.0) * H * dt;
  const double fv = (1.0 - xv) / (1.0 + xv);
  const double fE = (1.0 - xE) / (1.0 + xE);
  const double fe = (1.0 - xe) / (1.0 + xe);
  for (int64_t z = g; z < g + N[2]; ++z)
    for (int64_t y = g; y < g + N[1]; ++y)
      for (int64_t x = g; x < g + N[0]; ++x) {
        const int64_t o = (z * n[1] + y) * n[0] + x;
        G->vx[o] = G->vx[o] * fv;
        G->vy[o] = G->vy[o] * fv;
        G->vz[o] = G->vz[o] * fv;
        G->etot[o] = G->etot[o] * fE;
        G->eint[o] = G->eint[o] * fe;
      }
  return 0;
}

int ppmo_fill_periodic(ppmo_grid *G) {
  if (!G || G->nx < 1 || G->ny < 1 || G->nz < 1 || G->ghost < 0) return -1;
  const int g = G->ghost;
  const int N[3] = {G->nx, G->ny, G->nz};
  const int64_t n[3] = {N[0] + 2 * g, N[1] + 2 * g, N[2] + 2 * g};
  double *f[6] = {G->rho, G->vx, G->vy, G->vz, G->etot, G->eint};
  auto wrap = [&](int i, int d) { return g + (((i - g) % N[d]) + N[d]) % N[d]; };
  for (int k = 0; k < n[2]; ++k)
    for (int j = 0; j < n[1]; ++j)
      for (int i = 0; i < n[0]; ++i) {
        const int ii = wrap(i, 0), jj = wrap(j, 1), kk = wrap(k, 2);
        if (ii == i && jj == j && kk == k) continue;
        const int64_t dst = (k * n[1] + j) * n[0] + i, src = (kk * n[1] + jj) * n[0] + ii;
        for (int q = 0; q < 6; ++q) f[q][dst] = f[q][src];
      }
  return 0;
}

int ppmo_fill_boundary(ppmo_grid *G, const int32_t kinds[6], const double *inflow) {
  if (!G || !kinds || G->nx < 1 || G->ny < 1 || G->nz < 1 || G->ghost < 0) return -1;
  const int g = G->ghost;
  const int N[3] = {G->nx, G->ny, G->nz};
  for (int a = 0; a < 3; ++a) {
    for (int s = 0; s < 2; ++s) {
      const int k = kinds[2 * a + s];
      if (k < PPMO_FACE_PERIODIC || k > PPMO_FACE_INFLOW) return -1;
      if (k == PPMO_FACE_INFLOW && !inflow) return -1;
      if (k == PPMO_FACE_REFLECTING && N[a] < g) return -1;
    }
    if ((kinds[2 * a] == PPMO_FACE_PERIODIC) != (kinds[2 * a + 1] == PPMO_FACE_PERIODIC)) return -1;
  }
  const int64_t n[3] = {N[0] + 2 * g, N[1] + 2 * g, N[2] + 2 * g};
  double *f[6] = {G->rho, G->vx, G->vy, G->vz, G->etot, G->eint};
  // Axis by axis: axis a over its ghost layers, the axes before it over
  // their whole extent (ghosts already filled), the axes after it over their
  // active range.
  for (int a = 0; a < 3; ++a) {
    int lo[3], hi[3];
    for (int b = 0; b < 3; ++b) {
      lo[b] = b < a ? 0 : g;
      hi[b] = b < a ? int(n[b]) : g + N[b];
    }
    lo[a] = 0;
    hi[a] = int(n[a]);
    for (int z = lo[2]; z < hi[2]; ++z)
      for (int y = lo[1]; y < hi[1]; ++y)
        for (int x = lo[0]; x < hi[0]; ++x) {
          int c[3] = {x, y, z};
          const int ca = c[a];
          if (ca >= g && ca < g + N[a]) continue;  // active along a
          const int side = ca < g ? 0 : 1;
          const int kind = kinds[2 * a + side];
          const int64_t dst = (int64_t(z) * n[1] + y) * n[0] + x;
          if (kind == PPMO_FACE_INFLOW) {
            for (int q = 0; q < 6; ++q) f[q][dst] = inflow[(2 * a + side) * 6 + q];
            continue;
          }
          int sc;
          if (kind == PPMO_FACE_PERIODIC) sc = g + (((ca - g) % N[a]) + N[a]) % N[a];
          else if (kind == PPMO_FACE_REFLECTING) sc = side == 0 ? 2 * g - 1 - ca : 2 * (g + N[a]) - 1 - ca;
          else sc = side == 0 ? g : g + N[a] - 1;  // outflow: the edge cell
          c[a] = sc;
          const int64_t src = (int64_t(c[2]) * n[1] + c[1]) * n[0] + c[0];
          for (int q = 0; q < 6; ++q) f[q][dst] = f[q][src];
          if (kind == PPMO_FACE_REFLECTING) f[1 + a][dst] = -f[1 + a][src];
        }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// SecondOrderA interpolation (Appendix "Interpolation", three-dimensional
// form).  nb[dz][dy][dx] is the 3x3x3 neighbourhood of the coarse cell Q0 =
// nb[1][1][1]; out[k][j][i] receives the r^3 fine values it covers.
//  - The corner values Q_{sx,sy,sz} (s = -/+ 1/2) are the averages of the 8
//    coarse cells sharing the corner (added in increasing z, y, x).
//  - Limited slopes along the four diagonals (minmod of the two half-cell
//    differences): dQ0 from corner (-,-,-) to (+,+,+), dQ1 from (+,-,-) to
//    (-,+,+), dQ2 from (-,+,-) to (+,-,+), dQ3 from (-,-,+) to (+,+,-); these
//    are the diagonals for which the paper's conversion f_x = dQ2 + dQ3,
//    f_y = dQ1 + dQ3, f_z = dQ1 + dQ2 makes dQn the change from the centre
//    to the corner.
//  - A linear function's change to corner (+,+,+) is dQ1 + dQ2 + dQ3, so
//    s = (dQ1 + dQ2 + dQ3) / dQ0 must lie in [0, 1]; otherwise the slopes
//    that push it out (chi = 1: those opposite to dQ0 when s < 0, those along
//    dQ0 when s > 1) are scaled by f so that the sum becomes dQ0 * s' with
//    s' = min(max(s, 0), 1).  With dQ0 = 0 the sum must vanish: if it does
//    not, the slopes along its sign are scaled to make it zero.
//  - q(i,j,k) = Q0 + ((i + (1-r)/2)/r) f_x + ((j + (1-r)/2)/r) f_y
//    + ((k + (1-r)/2)/r) f_z.
void ppmo_second_order_a(const double *nb27, int32_t r, double *out) {
  double nb[3][3][3];
  for (int z = 0; z < 3; ++z)
    for (int y = 0; y < 3; ++y)
      for (int x = 0; x < 3; ++x) nb[z][y][x] = nb27[(z * 3 + y) * 3 + x];
  second_order_a<double>(nb, r, out);
}


// Ghost cells of a fine grid from its parent (Sec. "Boundary conditions":
// interpolation from the parent, conservative and monotonic): every cell of
// the fine grid outside its active region takes the SecondOrderA value of
// the conserved quantities rho, rho v, rho E, rho e of the parent cell that
// covers it; the velocities and specific energies are those over the
// interpolated density.
int ppmo_fill_from_parent(ppmo_grid *F, const int32_t fine_start[3], const ppmo_grid *C,
                          const int32_t parent_start[3], int32_t r) {
  if (!F || !C || !fine_start || !parent_start || r < 2) return -1;
  const int gf = F->ghost, gc = C->ghost;
  const int Nf[3] = {F->nx, F->ny, F->nz}, Nc[3] = {C->nx, C->ny, C->nz};
  const int64_t nf[3] = {Nf[0] + 2 * gf, Nf[1] + 2 * gf, Nf[2] + 2 * gf};
  const int64_t nc[3] = {Nc[0] + 2 * gc, Nc[1] + 2 * gc, Nc[2] + 2 * gc};
  // every coarse cell used, and its 27 neighbours, must lie in the parent array
  for (int a = 0; a < 3; ++a) {
    const int64_t lo = floor_div(fine_start[a] - gf, r) - parent_start[a] + gc;
    const int64_t hi = floor_div(fine_start[a] + Nf[a] + gf - 1, r) - parent_start[a] + gc;
    if (lo < 1 || hi > nc[a] - 2) return -1;
  }
  const double *cf[6] = {C->rho, C->vx, C->vy, C->vz, C->etot, C->eint};
  double *ff[6] = {F->rho, F->vx, F->vy, F->vz, F->etot, F->eint};
  // ghost cells are independent: threads over z planes, same result
#pragma omp parallel
  {
  std::vector<double> sub((size_t)r * r * r);
#pragma omp for schedule(static)
  for (int64_t z = 0; z < nf[2]; ++z)
    for (int64_t y = 0; y < nf[1]; ++y)
      for (int64_t x = 0; x < nf[0]; ++x) {
        const int64_t c[3] = {x, y, z};
        bool active = true;
        for (int a = 0; a < 3; ++a) active = active && c[a] >= gf && c[a] < gf + Nf[a];
        if (active) continue;
        int64_t lc[3];
        int si[3];
        for (int a = 0; a < 3; ++a) {
          const int64_t gfine = fine_start[a] + (c[a] - gf);
          const int64_t gcoarse = floor_div(gfine, r);
          si[a] = int(gfine - gcoarse * r);
          lc[a] = gcoarse - parent_start[a] + gc;
        }
        double q[6];
        for (int comp = 0; comp < 6; ++comp) {
          double nb[3][3][3];
          for (int dz = 0; dz < 3; ++dz)
            for (int dy = 0; dy < 3; ++dy)
              for (int dx = 0; dx < 3; ++dx) {
                const int64_t o = ((lc[2] + dz - 1) * nc[1] + (lc[1] + dy - 1)) * nc[0] +
                                  (lc[0] + dx - 1);
                nb[dz][dy][dx] = comp == 0 ? cf[0][o] : cf[0][o] * cf[comp][o];
              }
          second_order_a<double>(nb, r, sub.data());
          q[comp] = sub[((size_t)si[2] * r + si[1]) * r + si[0]];
        }
        const int64_t dst = (z * nf[1] + y) * nf[0] + x;
        ff[0][dst] = q[0];
        for (int comp = 1; comp < 6; ++comp) ff[comp][dst] = q[comp] / q[0];
      }
  }
  return 0;
}

// Sibling copy: every cell of dst outside its active region that lies in the
// active region of src (same level; starts are global indices of the first
// active cells) takes src's values.
int ppmo_copy_from_sibling(ppmo_grid *D, const int32_t dst_start[3], const ppmo_grid *S,
                           const int32_t src_start[3]) {
  if (!D || !S || !dst_start || !src_start) return -1;
  const int gd = D->ghost, gs = S->ghost;
  const int Nd[3] = {D->nx, D->ny, D->nz}, Ns[3] = {S->nx, S->ny, S->nz};
  const int64_t nd[3] = {Nd[0] + 2 * gd, Nd[1] + 2 * gd, Nd[2] + 2 * gd};
  const int64_t ns[3] = {Ns[0] + 2 * gs, Ns[1] + 2 * gs, Ns[2] + 2 * gs};
  const double *sf[6] = {S->rho, S->vx, S->vy, S->vz, S->etot, S->eint};
  double *df[6] = {D->rho, D->vx, D->vy, D->vz, D->etot, D->eint};
  // only dst cells whose image lies in src's active region can be copied:
  // local c with 0 <= dst_start + c - gd - src_start < Ns, within dst's array
  int64_t lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = std::max<int64_t>(0, (int64_t)src_start[a] - dst_start[a] + gd);
    hi[a] = std::min<int64_t>(nd[a], (int64_t)src_start[a] + Ns[a] - dst_start[a] + gd);
  }
  for (int64_t z = lo[2]; z < hi[2]; ++z)
    for (int64_t y = lo[1]; y < hi[1]; ++y)
      for (int64_t x = lo[0]; x < hi[0]; ++x) {
        const int64_t c[3] = {x, y, z};
        bool active = true, inside = true;
        int64_t sc[3];
        for (int a = 0; a < 3; ++a) {
          active = active && c[a] >= gd && c[a] < gd + Nd[a];
          const int64_t g = dst_start[a] + (c[a] - gd) - src_start[a];  // src active index
          inside = inside && g >= 0 && g < Ns[a];
          sc[a] = g + gs;
        }
        if (active || !inside) continue;
        const int64_t dst = (z * nd[1] + y) * nd[0] + x;
        const int64_t src = (sc[2] * ns[1] + sc[1]) * ns[0] + sc[0];
        for (int q = 0; q < 6; ++q) df[q][dst] = sf[q][src];
      }
  return 0;
}

void ppmo_two_shock(const ppmo_params *p, const double l[3], const double r[3], double out[7]) {
  RiemannOut<double> o = two_shock<double>(*p, l[0], l[1], l[2], r[0], r[1], r[2]);
  out[0] = o.ps; out[1] = o.us; out[2] = o.rho; out[3] = o.u; out[4] = o.p;
  out[5] = o.iters; out[6] = o.left ? 1.0 : 0.0;
}

void ppmo_hll_flux(const ppmo_params *p, const double l[5], const double r[5], double out[7]) {
  hll_flux<double>(*p, l, r, out);
}

void ppmo_hllc_flux(const ppmo_params *p, const double l[5], const double r[5], double out[7]) {
  hllc_flux<double>(*p, l, r, out);
}

int ppmo_count_ops(ppmo_grid *G, const ppmo_params *P, double dt, int32_t order,
                   int64_t ops[6]) {
  if (!valid_grid(G) || !valid_params(P) || order < 0 || order > 5 || !(dt > 0)) return -1;
  opc_reset();
  int64_t cells = 0;
  const int g = G->ghost;
  const int N[3] = {G->nx, G->ny, G->nz};
  int mask = 0;
  for (int s = 0; s < 3; ++s) {
    const int axis = kOrders[order][s];
    mask |= 1 << axis;
    const int am = mask & ~(1 << axis);
    int64_t c = N[axis];
    for (int d = 0; d < 3; ++d)
      if (d != axis) c *= (am >> d) & 1 ? N[d] : N[d] + 2 * g;
    cells += c;
  }
#ifdef _OPENMP
  int saved = omp_get_max_threads();
  omp_set_num_threads(1);
#endif
  step_impl<OpCount>(G, P, dt, order, nullptr);
#ifdef _OPENMP
  omp_set_num_threads(saved);
#endif
  opc_read(ops);
  ops[5] = cells;
  return 0;
}

int ppmo_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void ppmo_set_num_threads(int32_t n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

}  // extern "C"
