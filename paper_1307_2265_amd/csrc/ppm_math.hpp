// ppm_math.hpp -- per-cell and per-face arithmetic of the PPM sweep (device).
//
// Each function is one step of the direct-Eulerian PPM update of the Enzo
// method paper (Sec. "Hydrodynamics: The PPM method"), written for a single
// cell or face so that the sweep kernel can stream a pencil through them.
// The library is compiled with -ffp-contract=off and without fast-math: in
// double precision every expression below is evaluated exactly as written,
// operation by operation, so its result is fixed by IEEE-754 alone.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace ppm {

// Parabola coefficients (CW84 Eqs. 1.5-1.6 on a uniform grid).
constexpr double kC16 = 1.0 / 6.0;
constexpr double kC23 = 2.0 / 3.0;
// Contact steepening (CW84 Eqs. 1.16-1.17 and the contact test, Eq. 3.2).
constexpr double kSteepEps = 0.01;
constexpr double kSteepK0 = 0.1;
constexpr double kSteepEta1 = 20.0;
constexpr double kSteepEta2 = 0.05;
// Shock flattening (CW84 appendix).
constexpr double kFlatOmega1 = 0.75;
constexpr double kFlatOmega2 = 10.0;
constexpr double kFlatEps = 0.33;

enum : uint32_t {
  kSteepen = 1u, kFlatten = 2u, kDualEnergy = 4u, kFallbackHLL = 8u, kHLLC = 16u,
  kDiffusion = 32u
};
// CW84's dissipation coefficient K of the optional diffusive flux.
constexpr double kDiffK = 0.1;
// Set by the library, never by a caller: some patch carries an acceleration
// field, so the sweeps launch their build with the gravity source terms.
constexpr uint32_t kAnyGravity = 0x80000000u;

struct Params {
  double gamma, cfl, eta1, eta2, rho_floor, p_floor, e_floor, riemann_rtol;
  int32_t riemann_max_iter;
  uint32_t flags;
  // nullable: per level, the expansion factor a and its rate adot at the
  // level's half step (device memory); null is the static case a = 1
  const double *expand;
  // sqrt((gamma-1)/(2 gamma)): a shock wave's Lagrangian speed over the sound
  // one, W_s / C_s, as the star pressure falls to zero
  double shock_k0;
};

// Expansion factor of a level (1 without expansion factors).
__device__ __forceinline__ double expansion_a(const Params &P, int level) {
  return P.expand ? P.expand[2 * level] : 1.0;
}

template <class T> __device__ __forceinline__ T vmin(T a, T b) { return a < b ? a : b; }
template <class T> __device__ __forceinline__ T vmax(T a, T b) { return a > b ? a : b; }
template <class T> __device__ __forceinline__ T clamp01(T x) {
  return x < T(0) ? T(0) : (x > T(1) ? T(1) : x);
}

// Correctly rounded double quotient and square root for operands of
// ordinary magnitude.  Both refine the hardware reciprocal (square root) by
// Newton steps on fused multiply-adds and finish with one exact-remainder
// correction, which yields the IEEE round-to-nearest result (Markstein's
// theorem; the square root likewise).  They omit the operand scaling and
// special-value fix-ups that a general IEEE division or square root needs for
// operands within 2^768 of the overflow or underflow threshold, zeros,
// infinities and NaNs.  They serve only where the operands are bounded: the
// equation of state and the Riemann solvers take floored states (floors of
// at least 1e-100 are enforced at the interface), the Lagrangian wave speeds
// and the two-shock star density are positive and finite for such states, and
// the steepening and flattening ratios divide differences of floored cell
// values; with state magnitudes below 1e100 every operand there is far inside
// the range, and the results are bit for bit those of a / b and sqrt(x).  The
// characteristic tracing, whose reconstructed edge values no floor bounds
// (an edge density or pressure can be zero), uses xdiv / xsqrt instead.
__device__ __forceinline__ double ddiv(double a, double b) {
  double y = __builtin_amdgcn_rcp(b);
  double e = fma(-b, y, 1.0);
  y = fma(y, e, y);
  e = fma(-b, y, 1.0);
  y = fma(y, e, y);
  const double q = a * y;
  const double r = fma(-b, q, a);
  return fma(r, y, q);
}
__device__ __forceinline__ double dsqrt(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y;   // sqrt(x)
  double h = y * 0.5; // 1 / (2 sqrt(x))
  const double e = fma(-h, s, 0.5);
  s = fma(s, e, s);
  h = fma(h, e, h);
  double d = fma(-s, s, x);
  s = fma(d, h, s);
  d = fma(-s, s, x);
  return fma(d, h, s);
}

// Quotient, reciprocal and square root of the reconstruction and tracing
// stages: correctly rounded in double; in the float stages of the mixed
// precision the hardware reciprocal and square root (1 ulp), well inside
// that path's error budget.
template <class T> __device__ __forceinline__ T rdiv(T a, T b) { return ddiv(a, b); }
template <> __device__ __forceinline__ float rdiv<float>(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);
}
// IEEE quotient and square root for every operand (zeros, infinities and the
// extreme exponents included), for the characteristic tracing; in the float
// stages of the mixed precision the hardware reciprocal and square root.
template <class T> __device__ __forceinline__ T xdiv(T a, T b) { return a / b; }
template <> __device__ __forceinline__ float xdiv<float>(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);
}
template <class T> __device__ __forceinline__ T xsqrt(T a) { return __builtin_sqrt(a); }
template <> __device__ __forceinline__ float xsqrt<float>(float a) {
  return __builtin_amdgcn_sqrtf(a);
}

// a * b + c: in double two rounded operations, exactly the expression as
// written (the FP64 path reproduces the oracle bit for bit); in the float
// stages of the mixed precision one fused multiply-add.
template <class T> __device__ __forceinline__ T mad(T a, T b, T c) { return a * b + c; }
template <> __device__ __forceinline__ float mad<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

// The ratio test a/b > t of the selection rules, as a > t*b when b > 0 (every
// physical state) and as written otherwise; the quotient is formed only when
// some lane of the wave has b <= 0.
__device__ __forceinline__ bool ratio_above(double a, double b, double t) {
  if (__builtin_expect(b > 0.0, 1)) return a > t * b;
  return a / b > t;
}

// ---------------------------------------------------------------------------
// Pressure from the dual-energy selection rule (eta1) and the sound speed.
// Velocities in pencil order: normal u, then the two transverse components.
__device__ __forceinline__ double eos_pressure(const Params &P, double rho, double u, double v1,
                                               double v2, double E, double e) {
  const double g = P.gamma;
  double ke = 0.5 * (u * u + v1 * v1 + v2 * v2);
  double eps = E - ke;
  if ((P.flags & kDualEnergy) && !ratio_above(eps, E, P.eta1)) eps = e;
  double pp = (g - 1.0) * rho * eps;
  if (pp < P.p_floor) pp = P.p_floor;
  return pp;
}
__device__ __forceinline__ void eos(const Params &P, double rho, double u, double v1, double v2,
                                    double E, double e, double &p, double &c) {
  const double pp = eos_pressure(P, rho, u, v1, v2, E, e);
  p = pp;
  c = dsqrt(ddiv(P.gamma * pp, rho));
}
// The pressure (double, from the selection rule) and the sound speed in the
// reconstruction type T: for float, sqrt(g p / rho) with the float
// reciprocal and square root (p / rho stays in range at the floors).
template <class T>
__device__ __forceinline__ void eos_cell(const Params &P, double rho, double u, double v1,
                                         double v2, double E, double e, double &p, T &c) {
  if constexpr (sizeof(T) == sizeof(double)) {
    double cd;
    eos(P, rho, u, v1, v2, E, e, p, cd);
    c = cd;
  } else {
    p = eos_pressure(P, rho, u, v1, v2, E, e);
    c = __builtin_amdgcn_sqrtf(float(P.gamma) * float(p) * __builtin_amdgcn_rcpf(float(rho)));
  }
}

// CW84 limited slope of a cell from its two neighbours.
template <class T> __device__ __forceinline__ T limited_slope(T qm, T q0, T qp) {
  T dl = q0 - qm, dr = qp - q0;
  T dc = T(0.5) * (qp - qm);
  T m = T(0);
  if (dl * dr > T(0)) {
    m = fabs(dc);
    if (T(2) * fabs(dl) < m) m = T(2) * fabs(dl);
    if (T(2) * fabs(dr) < m) m = T(2) * fabs(dr);
    if (dc < T(0)) m = -m;
  }
  return m;
}

// Fourth-order interface value between two cells from their limited slopes.
template <class T> __device__ __forceinline__ T interface_value(T q0, T q1, T dm0, T dm1) {
  return mad<T>(T(-kC16), dm1 - dm0, T(0.5) * (q0 + q1));
}

// Second difference of the density centred on a cell.
template <class T> __device__ __forceinline__ T second_diff(T qm, T q0, T qp) {
  return mad<T>(T(-2), q0, qp) + qm;
}

// Contact-steepening weight eta of a cell (0 = no steepening).
// rm/rp, pm/pp: density and pressure of the two neighbours; d2m/d2p: second
// differences centred on the two neighbours.
template <class T>
__device__ __forceinline__ T steepen_eta(double g, T rm, T rp, T pm, T pp, T d2m, T d2p) {
  T drho = rp - rm;
  T eta = T(0);
  if (d2p * d2m < T(0) && fabs(drho) - T(kSteepEps) * vmin<T>(fabs(rp), fabs(rm)) > T(0) &&
      T(g * kSteepK0) * fabs(drho) * vmin<T>(pp, pm) >= fabs(pp - pm) * vmin<T>(rp, rm)) {
    T etat = rdiv<T>(-(d2p - d2m), T(6) * drho);
    eta = clamp01<T>(T(kSteepEta1) * (etat - T(kSteepEta2)));
  }
  return eta;
}

// Flattening indicator f~ of a cell from the pressures two cells either side
// and the velocities of its neighbours.
template <class T>
__device__ __forceinline__ T flatten_indicator(T pm2, T pm1, T pp1, T pp2, T um1, T up1) {
  T dp = pp1 - pm1;
  T f = T(0);
  if (fabs(dp) > T(kFlatEps) * vmin<T>(pp1, pm1) && um1 - up1 > T(0)) {
    T den = pp2 - pm2;
    if (den == T(0)) f = T(1);
    else f = clamp01<T>(T(kFlatOmega2) * (rdiv<T>(dp, den) - T(kFlatOmega1)));
  }
  return f;
}

// CW84 Eq. 1.10: make the parabola monotone, then return Delta q and q_6.
template <class T> __device__ __forceinline__ void monotonize(T q, T &l, T &r, T &dq, T &q6) {
  if ((r - q) * (q - l) <= T(0)) {
    l = q;
    r = q;
  } else {
    T d = r - l;
    T s = d * mad<T>(T(-0.5), l + r, q);
    T d2 = d * d * T(kC16);
    if (s > d2) l = mad<T>(T(-2), r, T(3) * q);
    else if (-d2 > s) r = mad<T>(T(-2), l, T(3) * q);
  }
  dq = r - l;
  q6 = T(6) * mad<T>(T(-0.5), l + r, q);
}

// Average of the parabola over the right-edge domain of a right-moving wave
// of Courant number y, and over the left-edge domain of a left-moving one.
template <class T> __device__ __forceinline__ T avg_right(T qr, T dq, T q6, T y) {
  const T a = mad<T>(T(-kC23), y, T(1));
  return mad<T>(-(T(0.5) * y), mad<T>(-a, q6, dq), qr);
}
template <class T> __device__ __forceinline__ T avg_left(T ql, T dq, T q6, T y) {
  const T a = mad<T>(T(-kC23), y, T(1));
  return mad<T>(T(0.5) * y, mad<T>(a, q6, dq), ql);
}

// A cell's parabola for the five reconstructed quantities.
template <class T> struct Parabola {
  T l[5], dq[5], q6[5];  // left edge value, Delta q, q_6; r = l + dq
};

// Traced interface state (rho, u, v1, v2, p).
template <class T> struct State {
  T r, u, v1, v2, p;
};

// CW84 characteristic tracing (Eqs. 3.5-3.7) of one cell edge.
// RightEdge: the left state of the face to the right of the cell, built from
// the waves moving right (u-c, u, u+c > 0); the reference state is the
// average over the u+c domain, so the u+c correction vanishes whenever the
// sound speed of the edge state is positive and finite; it is still formed as
// the general formula writes it, which gives a NaN, not zero, when the edge
// density or pressure is zero.  Left edge: the mirror image, with the u-c
// domain as reference.
// q: cell-centre u; c: sound speed; lam = dt/dx.
template <class T, bool RightEdge>
__device__ __forceinline__ State<T> trace_edge(double g, const T (&ql)[5], const T (&qrr)[5],
                                               const T (&dq)[5], const T (&q6)[5], T u, T c,
                                               T lam, T rho_floor, T p_floor) {
  // quantity indices: 0 rho, 1 u, 2 v1, 3 v2, 4 p
  State<T> s;
  T yref, yslow, y0;
  if (RightEdge) {
    yslow = clamp01<T>((u - c) * lam);
    y0 = clamp01<T>(u * lam);
    yref = clamp01<T>((u + c) * lam);
  } else {
    yslow = clamp01<T>(-(u + c) * lam);
    y0 = clamp01<T>(-u * lam);
    yref = clamp01<T>(-(u - c) * lam);
  }
  auto avg = [&](int k, T y) -> T {
    return RightEdge ? avg_right<T>(qrr[k], dq[k], q6[k], y) : avg_left<T>(ql[k], dq[k], q6[k], y);
  };
  T rt = avg(0, yref), ut = avg(1, yref), pt = avg(4, yref);
  T C, iC, irt;
  if constexpr (sizeof(T) == sizeof(double)) {
    C = xsqrt<T>(T(g) * pt * rt);
    iC = xdiv<T>(T(1), C);
    irt = xdiv<T>(T(1), rt);
  } else {
    // float: C = rho sqrt(g p / rho) and 1/C = (1/rho) / sqrt(g p / rho), so
    // that no product of two edge values (each as small as the floors, whose
    // product lies below the float range) is formed
    irt = xdiv<T>(T(1), rt);
    const T c2 = T(g) * pt * irt;
    const T ic = __builtin_amdgcn_rsqf(c2);
    C = rt * (c2 * ic);
    iC = irt * ic;
  }
  // bref: the reference wave's own correction (its averages are ut, pt);
  // bslow: the other acoustic wave; b0: the entropy wave
  T bref = T(0), bslow = T(0), b0 = T(0);
  const bool ref_on = RightEdge ? (u + c > T(0)) : (u - c < T(0));
  const bool slow_on = RightEdge ? (u - c > T(0)) : (u + c < T(0));
  const bool zero_on = RightEdge ? (u > T(0)) : (u < T(0));
  if (ref_on) {
    if (RightEdge) bref = T(-0.5) * iC * ((ut - ut) + (pt - pt) * iC);        // beta-plus
    else bref = T(0.5) * iC * ((ut - ut) - (pt - pt) * iC);                   // beta-minus
  }
  if (slow_on) {
    T us = avg(1, yslow), ps = avg(4, yslow);
    if (RightEdge) bslow = T(0.5) * iC * mad<T>(-(pt - ps), iC, ut - us);     // beta-minus
    else bslow = T(-0.5) * iC * mad<T>(pt - ps, iC, ut - us);                  // beta-plus
  }
  if (zero_on) {
    T r0 = avg(0, y0), p0 = avg(4, y0);
    b0 = mad<T>((pt - p0) * iC, iC, irt) - xdiv<T>(T(1), r0);
  }
  T bp = RightEdge ? bref : bslow;
  T bm = RightEdge ? bslow : bref;
  T ps;
  if constexpr (sizeof(T) == sizeof(double)) ps = mad<T>(C * C, bp + bm, pt);
  else ps = mad<T>(C, C * (bp + bm), pt);  // C^2 alone can lie below the float range
  T us = mad<T>(C, bp - bm, ut);
  T tau = irt - (bp + bm + b0);
  T rs = tau > T(0) ? xdiv<T>(T(1), tau) : rt;
  s.r = vmax<T>(rs, rho_floor);
  s.u = us;
  s.p = vmax<T>(ps, p_floor);
  s.v1 = avg(2, y0);
  s.v2 = avg(3, y0);
  return s;
}

// Face flux in the flux type T of a precision: the mass and momentum fluxes
// F_rho, F_u, F_v1, F_v2 (pencil order), the internal-energy flux F_e and the
// face velocity of the p div v term in T, the total-energy flux F_E always in
// double.  get/set address the six fluxes and the face velocity by slot
// (0..3 mass and momenta, 4 F_E, 5 F_e, 6 the face velocity), in double.
template <class T> struct FluxT {
  T m[4];
  double E;
  T e;
  T ub;
  __device__ __forceinline__ double get(int k) const {
    return k < 4 ? double(m[k]) : (k == 4 ? E : (k == 5 ? double(e) : double(ub)));
  }
  __device__ __forceinline__ void set(int k, double v) {
    if (k < 4) m[k] = T(v);
    else if (k == 4) E = v;
    else if (k == 5) e = T(v);
    else ub = T(v);
  }
};
using Flux = FluxT<double>;

template <class T> __device__ __forceinline__ FluxT<T> zero_flux() {
  FluxT<T> F;
#pragma unroll
  for (int k = 0; k < 7; ++k) F.set(k, 0.0);
  return F;
}

// A double flux in the flux type T (the fallback's and HLLC's fluxes in the
// mixed precision).
template <class T> __device__ __forceinline__ FluxT<T> narrow_flux(const Flux &D) {
  FluxT<T> F;
#pragma unroll
  for (int k = 0; k < 7; ++k) F.set(k, D.get(k));
  return F;
}

// Two-shock Riemann solver (Sec. "Riemann Solvers and Fallback"), sampled at
// x/t = 0, and the fluxes of the sampled state.  Newton iteration on
// u*_R(p) - u*_L(p) = 0 with the Lagrangian shock speeds W_s.
// Star pressure of the two-shock problem: Newton iteration on
// u*_R(p) - u*_L(p) = 0 with the Lagrangian shock speeds W_s, from the
// acoustic guess, until the correction falls below rtol*p; the star state is
// that last iterate, whose shock speeds are already at hand.  Returns p* and
// the shock speeds, their reciprocals and the two sides' u* at p*.
struct StarState {
  double ps, wl, wr, iwl, iwr, usl, usr;
  int iters;
};
__device__ __forceinline__ StarState two_shock_star(const Params &P, double rl, double ul,
                                                    double pl, double rr, double ur,
                                                    double pr) {
  const double g = P.gamma;
  const double G1 = (g + 1.0) / (2.0 * g);
  double cl = dsqrt(g * pl * rl);
  double cr = dsqrt(g * pr * rr);
  double ipl = ddiv(1.0, pl), ipr = ddiv(1.0, pr);
  double ps = ddiv(cr * pl + cl * pr - cl * cr * (ur - ul), cl + cr);
  if (ps < P.p_floor) ps = P.p_floor;
  int it = 0;
  bool capped = false;
  double wl, wr, iwl, iwr, usl, usr;
  for (;;) {
    wl = cl * dsqrt(1.0 + G1 * (ps * ipl - 1.0));
    wr = cr * dsqrt(1.0 + G1 * (ps * ipr - 1.0));
    iwl = ddiv(1.0, wl);
    iwr = ddiv(1.0, wr);
    usl = ul - (ps - pl) * iwl;
    usr = ur + (ps - pr) * iwr;
    if (capped || it == P.riemann_max_iter) break;
    double izl = (wl * wl + cl * cl) * (0.5 * iwl * iwl * iwl);
    double izr = (wr * wr + cr * cr) * (0.5 * iwr * iwr * iwr);
    double pn = ps - ddiv(usr - usl, izl + izr);
    if (pn < P.p_floor) pn = P.p_floor;
    ++it;
    if (fabs(pn - ps) <= P.riemann_rtol * pn) break;
    ps = pn;
    if (it == P.riemann_max_iter) capped = true;
  }
  return StarState{ps, wl, wr, iwl, iwr, usl, usr, it};
}

__device__ __forceinline__ Flux two_shock_flux(const Params &P, double rl, double ul, double v1l,
                                               double v2l, double pl, double rr, double ur,
                                               double v1r, double v2r, double pr, int &iters) {
  const double g = P.gamma;
  const StarState st = two_shock_star(P, rl, ul, pl, rr, ur, pr);
  const double ps = st.ps, wl = st.wl, wr = st.wr, iwl = st.iwl, iwr = st.iwr;
  const double usl = st.usl, usr = st.usr;
  const int it = st.iters;
  iters = it;
  double us = 0.5 * (usl + usr);
  // sample the upwind side of the contact at x/t = 0
  const bool left = us >= 0.0;
  double rK = left ? rl : rr, uK = left ? ul : ur, pK = left ? pl : pr;
  double iwK = left ? iwl : iwr;
  double rs = ddiv(1.0, ddiv(1.0, rK) - (ps - pK) * iwK * iwK);
  if (rs < P.rho_floor) rs = P.rho_floor;
  // the upwind side's waves move away from the face: u - (speed) on the
  // left, u + (speed) on the right.  Written once with the side's values
  // and sign (x - y is x + (-y) exactly, and -h / (t - h) = h / (h - t)
  // exactly), so a wave whose lanes sample both sides evaluates each
  // division and square root once.
  const double sgn = left ? -1.0 : 1.0;
  const double wK = left ? wl : wr;
  double rb, ub, pb;
  if (ps > pK) {  // shock on the upwind side
    const double sK = uK + sgn * ddiv(wK, rK);
    const bool keep = left ? sK >= 0.0 : sK <= 0.0;
    if (keep) { rb = rK; ub = uK; pb = pK; }
    else { rb = rs; ub = us; pb = ps; }
  } else {        // rarefaction: linear through the fan
    const double head = uK + sgn * dsqrt(ddiv(g * pK, rK));
    const double tail = us + sgn * dsqrt(ddiv(g * ps, rs));
    bool outside = left ? head >= 0.0 : head <= 0.0;
    bool star = left ? tail <= 0.0 : tail >= 0.0;
    if (outside) { rb = rK; ub = uK; pb = pK; }
    else if (star) { rb = rs; ub = us; pb = ps; }
    else {
      double w = ddiv(-head, tail - head);
      rb = (1.0 - w) * rK + w * rs;
      ub = (1.0 - w) * uK + w * us;
      pb = (1.0 - w) * pK + w * ps;
    }
  }
  double v1 = left ? v1l : v1r;
  double v2 = left ? v2l : v2r;
  Flux F;
  double fr = rb * ub;
  F.m[0] = fr;
  F.m[1] = fr * ub + pb;
  F.m[2] = fr * v1;
  F.m[3] = fr * v2;
  double eb = ddiv(pb, (g - 1.0) * rb);
  double Eb = eb + 0.5 * (ub * ub + v1 * v1 + v2 * v2);
  F.E = fr * Eb + ub * pb;
  F.e = fr * eb;
  F.ub = ub;
  return F;
}

// Double reciprocal and reciprocal square root to about an ulp: the
// hardware estimates refined by two Newton steps (fused multiply-adds).
// For the mixed precision's double arithmetic, which needs double accuracy
// but not the correctly rounded results of the FP64 path.
__device__ __forceinline__ double rcp64(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ double rsqrt64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = fma(y, fma(-h * y, y, 0.5), y);
  return fma(y, fma(-h * y, y, 0.5), y);
}
// The same with one Newton step: the hardware estimates carry about 24
// correct bits, so the result is good to about 2^-47 -- ample where the value
// feeds an iteration that corrects it or a float result.
__device__ __forceinline__ double rcp64_1(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return fma(y, fma(-x, y, 1.0), y);
}
__device__ __forceinline__ double rsqrt64_1(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return fma(y, fma(-(0.5 * x) * y, y, 0.5), y);
}

// Star pressure of the two-shock problem for the mixed precision, in double
// with the same iteration, stopping rule and cap as two_shock_star (from a
// better start on expanding faces, below): with
// X = 1 + (g+1)/(2g) (p/p_s - 1) and y = 1/sqrt(X), the Lagrangian speed is
// W_s = C_s X y, 1/W_s = y / C_s, and Newton's step needs 1/Z_s =
// (W_s^2 + C_s^2) / (2 W_s^3) = (1 + y^2) / (2 W_s), so an iteration takes one
// reciprocal square root per side and one reciprocal, each good to about
// 2^-47 (the iteration converges to the root of the function so evaluated,
// within a few 1e-15 of the exact one).
__device__ __forceinline__ StarState two_shock_star_mixed(const Params &P, double rl, double ul,
                                                          double pl, double rr, double ur,
                                                          double pr) {
  const double g = P.gamma;
  const double G1 = (g + 1.0) / (2.0 * g);
  const double al = g * pl * rl, ar = g * pr * rr;
  const double icl = rsqrt64_1(al), icr = rsqrt64_1(ar);
  const double cl = al * icl, cr = ar * icr;
  const double ipl = rcp64_1(pl), ipr = rcp64_1(pr);
  const double iden = rcp64_1(cl + cr);
  double ps = (cr * pl + cl * pr - cl * cr * (ur - ul)) * iden;
  // Below the smaller side pressure the acoustic guess (impedances C_s) is far
  // from the root of a strongly expanding face, often negative; start from
  // the same linear estimate with the impedances the shock relation gives as
  // p -> 0, W_s = k0 C_s, capped at that pressure.  Converges to the same
  // star pressure, in fewer steps on the wave's slowest faces.
  const double pmin = pl < pr ? pl : pr;
  if (ps < pmin) {
    const double ex = (cr * pl + cl * pr - P.shock_k0 * (cl * cr * (ur - ul))) * iden;
    ps = ex < pmin ? ex : pmin;
  }
  if (ps < P.p_floor) ps = P.p_floor;
  int it = 0;
  bool capped = false;
  double wl, wr, iwl, iwr, usl, usr, yl, yr;
  for (;;) {
    const double xl = fma(G1, fma(ps, ipl, -1.0), 1.0);
    const double xr = fma(G1, fma(ps, ipr, -1.0), 1.0);
    yl = rsqrt64_1(xl);
    yr = rsqrt64_1(xr);
    wl = cl * (xl * yl);
    wr = cr * (xr * yr);
    iwl = icl * yl;
    iwr = icr * yr;
    usl = fma(-(ps - pl), iwl, ul);
    usr = fma(ps - pr, iwr, ur);
    if (capped || it == P.riemann_max_iter) break;
    const double izl = fma(yl, yl, 1.0) * (0.5 * iwl);
    const double izr = fma(yr, yr, 1.0) * (0.5 * iwr);
    double pn = fma(-(usr - usl), rcp64_1(izl + izr), ps);
    if (pn < P.p_floor) pn = P.p_floor;
    ++it;
    if (fabs(pn - ps) <= P.riemann_rtol * pn) break;
    ps = pn;
    if (it == P.riemann_max_iter) capped = true;
  }
  return StarState{ps, wl, wr, iwl, iwr, usl, usr, it};
}

// Two-shock flux of the mixed precision: the traced states come in float; the
// star pressure is iterated in double (two_shock_star_mixed); the sampling of the
// solution at x/t = 0 and the mass, momentum and internal-energy fluxes are
// formed in float (hardware reciprocal and square root), the total-energy
// flux in double from the sampled float state.
__device__ __forceinline__ FluxT<float> two_shock_flux_mixed(const Params &P, float rl, float ul,
                                                             float v1l, float v2l, float pl,
                                                             float rr, float ur, float v1r,
                                                             float v2r, float pr) {
  const StarState st = two_shock_star_mixed(P, double(rl), double(ul), double(pl), double(rr),
                                            double(ur), double(pr));
  const float g = float(P.gamma);
  const float ps = float(st.ps);
  const float us = float(0.5 * (st.usl + st.usr));
  const bool left = us >= 0.0f;
  const float rK = left ? rl : rr, uK = left ? ul : ur, pK = left ? pl : pr;
  const float wK = float(left ? st.wl : st.wr), iwK = float(left ? st.iwl : st.iwr);
  const float irK = __builtin_amdgcn_rcpf(rK);
  float rs = __builtin_amdgcn_rcpf(__builtin_fmaf(-(ps - pK) * iwK, iwK, irK));
  if (rs < float(P.rho_floor)) rs = float(P.rho_floor);
  float rb, ub, pb;
  if (ps > pK) {  // shock on the upwind side: its speed u_K -+ W_K / rho_K
    const float S = __builtin_fmaf(left ? -wK : wK, irK, uK);
    const bool keep = left ? S >= 0.0f : S <= 0.0f;
    if (keep) { rb = rK; ub = uK; pb = pK; }
    else { rb = rs; ub = us; pb = ps; }
  } else {        // rarefaction: linear through the fan
    const float cK = __builtin_amdgcn_sqrtf(g * pK * irK);
    const float cs = __builtin_amdgcn_sqrtf(g * ps * __builtin_amdgcn_rcpf(rs));
    const float head = left ? uK - cK : uK + cK;
    const float tail = left ? us - cs : us + cs;
    const bool outside = left ? head >= 0.0f : head <= 0.0f;
    const bool star = left ? tail <= 0.0f : tail >= 0.0f;
    if (outside) { rb = rK; ub = uK; pb = pK; }
    else if (star) { rb = rs; ub = us; pb = ps; }
    else {
      const float w = head * __builtin_amdgcn_rcpf(head - tail);
      rb = __builtin_fmaf(w, rs - rK, rK);
      ub = __builtin_fmaf(w, us - uK, uK);
      pb = __builtin_fmaf(w, ps - pK, pK);
    }
  }
  const float v1 = left ? v1l : v1r;
  const float v2 = left ? v2l : v2r;
  FluxT<float> F;
  const float fr = rb * ub;
  F.m[0] = fr;
  F.m[1] = __builtin_fmaf(fr, ub, pb);
  F.m[2] = fr * v1;
  F.m[3] = fr * v2;
  F.e = fr * (pb * __builtin_amdgcn_rcpf((g - 1.0f) * rb));
  F.ub = ub;
  // total energy flux in double: rho u is exact in double for float factors
  const double rbd = rb, ubd = ub, pbd = pb, v1d = v1, v2d = v2;
  const double frd = rbd * ubd;
  const double eb = pbd * rcp64((P.gamma - 1.0) * rbd);
  F.E = frd * (eb + 0.5 * (ubd * ubd + v1d * v1d + v2d * v2d)) + ubd * pbd;
  return F;
}

// HLLC flux (Sec. "Riemann Solvers and Fallback": HLL with the contact wave
// restored), the solver kHLLC selects in place of two-shock.  Outer wave
// speeds are the Davis estimates of the HLL fallback; the contact speed S*
// follows from the Rankine-Hugoniot conditions across the two outer waves
// with a common pressure and normal velocity at the contact; between outer
// wave s_K and the contact the state is rho*_K = rho_K (s_K - u_K)/(s_K - S*),
// u = S*, the transverse velocities and internal energy of side K, and
// E*_K = E_K + (S* - u_K)(S* + p_K / (rho_K (s_K - u_K))).  The flux at
// x/t = 0 is that of the upwind side, F_K + s_K (U*_K - U_K) inside the fan;
// the face velocity slot carries S*.
__device__ __forceinline__ Flux hllc_flux(const Params &P, double rl, double ul, double v1l,
                                          double v2l, double pl, double rr, double ur,
                                          double v1r, double v2r, double pr) {
  const double g = P.gamma;
  const double cl = dsqrt(ddiv(g * pl, rl)), cr = dsqrt(ddiv(g * pr, rr));
  const double el = ddiv(pl, (g - 1.0) * rl), er = ddiv(pr, (g - 1.0) * rr);
  const double El = el + 0.5 * (ul * ul + v1l * v1l + v2l * v2l);
  const double Er = er + 0.5 * (ur * ur + v1r * v1r + v2r * v2r);
  const double sL = vmin<double>(ul - cl, ur - cr);
  const double sR = vmax<double>(ul + cl, ur + cr);
  const bool fan = !(sL >= 0.0) && !(sR <= 0.0);
  double S = 0.0;
  bool left = sL >= 0.0;
  if (fan) {
    const double ml = rl * (sL - ul), mr = rr * (sR - ur);
    S = ddiv(pr - pl + ml * ul - mr * ur, ml - mr);
    left = S >= 0.0;
  }
  const double rK = left ? rl : rr, uK = left ? ul : ur, pK = left ? pl : pr;
  const double v1K = left ? v1l : v1r, v2K = left ? v2l : v2r;
  const double EK = left ? El : Er, eK = left ? el : er, sK = left ? sL : sR;
  const double fr = rK * uK;
  Flux F;
  F.m[0] = fr;
  F.m[1] = fr * uK + pK;
  F.m[2] = fr * v1K;
  F.m[3] = fr * v2K;
  F.E = uK * (rK * EK + pK);
  F.e = fr * eK;
  F.ub = uK;
  if (!fan) return F;
  const double mK = rK * (sK - uK);
  const double rs = ddiv(mK, sK - S);
  F.m[0] = F.m[0] + sK * (rs - rK);
  F.m[1] = F.m[1] + sK * (rs * S - rK * uK);
  F.m[2] = F.m[2] + sK * (rs * v1K - rK * v1K);
  F.m[3] = F.m[3] + sK * (rs * v2K - rK * v2K);
  F.E = F.E + sK * (rs * (EK + (S - uK) * (S + ddiv(pK, mK))) - rK * EK);
  F.e = F.e + sK * (rs * eK - rK * eK);
  F.ub = S;
  return F;
}

// The face flux of the solver a kernel is built for: two-shock, or HLLC
// (the flag kHLLC picks the kernel build at launch, so the two solvers'
// launches are separate kernels).  The HLLC build keeps the two-shock path
// behind the same flag: without it the FP64 marching loop is allocated with
// 44 spilled registers instead of 16 and runs 30 % slower (measured).
template <bool kUseHLLC>
__device__ __forceinline__ Flux riemann_flux(const Params &P, double rl, double ul, double v1l,
                                             double v2l, double pl, double rr, double ur,
                                             double v1r, double v2r, double pr) {
  if (kUseHLLC && (P.flags & kHLLC)) {
    return hllc_flux(P, rl, ul, v1l, v2l, pl, rr, ur, v1r, v2r, pr);
  } else {
    int iters;
    return two_shock_flux(P, rl, ul, v1l, v2l, pl, rr, ur, v1r, v2r, pr, iters);
  }
}

// The face flux of the solver a kernel is built for, in the flux type of
// its precision: the double solvers above for FP64; in the mixed precision
// the two-shock flux of the mixed form, and HLLC (kept in double) narrowed.
template <bool kUseHLLC, class T>
__device__ __forceinline__ FluxT<T> face_flux(const Params &P, const State<T> &l,
                                              const State<T> &r) {
  if constexpr (sizeof(T) == sizeof(double)) {
    return riemann_flux<kUseHLLC>(P, l.r, l.u, l.v1, l.v2, l.p, r.r, r.u, r.v1, r.v2, r.p);
  } else {
    if (kUseHLLC && (P.flags & kHLLC))
      return narrow_flux<T>(hllc_flux(P, double(l.r), double(l.u), double(l.v1), double(l.v2),
                                      double(l.p), double(r.r), double(r.u), double(r.v1),
                                      double(r.v2), double(r.p)));
    return two_shock_flux_mixed(P, l.r, l.u, l.v1, l.v2, l.p, r.r, r.u, r.v1, r.v2, r.p);
  }
}

// HLL flux with Davis wave speeds (the fallback solver).
__device__ __forceinline__ Flux hll_flux(const Params &P, const double (&sl)[5],
                                         const double (&sr)[5]) {
  const double g = P.gamma;
  double rl = sl[0], ul = sl[1], pl = sl[4];
  double rr = sr[0], ur = sr[1], pr = sr[4];
  double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
  double el = pl / ((g - 1.0) * rl), er = pr / ((g - 1.0) * rr);
  double El = el + 0.5 * (ul * ul + sl[2] * sl[2] + sl[3] * sl[3]);
  double Er = er + 0.5 * (ur * ur + sr[2] * sr[2] + sr[3] * sr[3]);
  double Ul[6] = {rl, rl * ul, rl * sl[2], rl * sl[3], rl * El, rl * el};
  double Ur[6] = {rr, rr * ur, rr * sr[2], rr * sr[3], rr * Er, rr * er};
  double Fl[6] = {rl * ul, rl * ul * ul + pl, rl * ul * sl[2], rl * ul * sl[3],
                  ul * (rl * El + pl), rl * ul * el};
  double Fr[6] = {rr * ur, rr * ur * ur + pr, rr * ur * sr[2], rr * ur * sr[3],
                  ur * (rr * Er + pr), rr * ur * er};
  double sL = vmin<double>(ul - cl, ur - cr);
  double sR = vmax<double>(ul + cl, ur + cr);
  Flux F;
  if (sL >= 0.0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) F.set(k, Fl[k]);
    F.ub = ul;
  } else if (sR <= 0.0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) F.set(k, Fr[k]);
    F.ub = ur;
  } else {
    double id = 1.0 / (sR - sL);
#pragma unroll
    for (int k = 0; k < 6; ++k)
      F.set(k, (sR * Fl[k] - sL * Fr[k] + sL * sR * (Ur[k] - Ul[k])) * id);
    double um_r = (sR * Ur[0] - sL * Ul[0] - (Fr[0] - Fl[0])) * id;
    double um_m = (sR * Ur[1] - sL * Ul[1] - (Fr[1] - Fl[1])) * id;
    F.ub = um_m / um_r;
  }
  return F;
}

// Optional diffusive flux of CW84 along the sweep: where the flow converges
// across the face (u_l > u_r, the two cells' normal velocities at the sweep
// input), each conserved quantity's flux gains nu (Q_l - Q_r), nu = K (u_l -
// u_r), Q = rho, rho u, rho v1, rho v2, rho E, rho e; the face velocity of the
// p div v term is left alone.
template <class T>
__device__ __forceinline__ void add_diffusion(FluxT<T> &F, double rl, double ul, double v1l,
                                              double v2l, double El, double el, double rr,
                                              double ur, double v1r, double v2r, double Er,
                                              double er) {
  const double du = ul - ur;
  if (!(du > 0.0)) return;
  const double nu = kDiffK * du;
  const double ql[6] = {rl, rl * ul, rl * v1l, rl * v2l, rl * El, rl * el};
  const double qr[6] = {rr, rr * ur, rr * v1r, rr * v2r, rr * Er, rr * er};
#pragma unroll
  for (int k = 0; k < 6; ++k) F.set(k, F.get(k) + nu * (ql[k] - qr[k]));
}

// Sweep-input state of a cell as the update needs it: density and velocity
// in the flux type T (as stored), energies, pressure and the eta2
// neighbourhood maximum in double.
template <class T> struct CellInT {
  T rho, u, v1, v2;
  double E, e, p, rhoEmax;
};
using CellIn = CellInT<double>;

// Conservative update of one cell from its two face fluxes (Eqs. mass_diff,
// momentum_diff, energy_diff, gasenergy_diff with the flux difference taken
// with a minus sign; lam = dt / (a dx) in comoving coordinates), then the
// eta2 resync (Eq. dualselect).  With a gravity field (grav), the
// time-centred sources of Eqs. momentum_diff and energy_diff: momentum gains
// hg (rho^n + rho^{n+1}) and total energy hg (rho^n u^n + rho^{n+1} u^{n+1}),
// where hg = (dt / 2) g / a with g the acceleration along the sweep at the
// cell centre.  Returns true when the new density or the eta1-selected
// internal energy is not positive.
__device__ __forceinline__ bool update_cell(const Params &P, double lam, const CellIn &c,
                                            const Flux &Fm, const Flux &Fp, double (&out)[6],
                                            bool grav = false, double hg = 0.0) {
  const bool dual = (P.flags & kDualEnergy) != 0;
  double rn = c.rho - lam * (Fp.m[0] - Fm.m[0]);
  double mu = c.rho * c.u - lam * (Fp.m[1] - Fm.m[1]);
  double m1 = c.rho * c.v1 - lam * (Fp.m[2] - Fm.m[2]);
  double m2 = c.rho * c.v2 - lam * (Fp.m[3] - Fm.m[3]);
  double mE = c.rho * c.E - lam * (Fp.E - Fm.E);
  double me = c.rho * c.e - lam * (Fp.e - Fm.e) - lam * c.p * (Fp.ub - Fm.ub);
  if (grav) {
    mu = mu + hg * (c.rho + rn);
    mE = mE + hg * (c.rho * c.u + mu);
  }
  double ir = ddiv(1.0, rn);
  double un = mu * ir, v1n = m1 * ir, v2n = m2 * ir, En = mE * ir, eraw = me * ir;
  double ke = 0.5 * (un * un + v1n * v1n + v2n * v2n);
  double epsE = En - ke;
  bool bad = !(rn > P.rho_floor);
  double sel = epsE;
  if (dual && !ratio_above(epsE, En, P.eta1)) sel = eraw;
  if (!(sel > 0.0)) bad = true;
  double en = eraw < P.e_floor ? P.e_floor : eraw;
  if (dual && ratio_above(rn * epsE, c.rhoEmax, P.eta2)) en = epsE;
  out[0] = rn; out[1] = un; out[2] = v1n; out[3] = v2n; out[4] = En; out[5] = en;
  return bad;
}

// The update of the mixed precision: density and momenta from the float
// fluxes in float, the velocities by the float reciprocal of the new density;
// total and internal energy accumulated in double (the energy fluxes, the
// p div v term and the division by the new density in double), the
// dual-energy selection (eta1) and resync (eta2) in double.
__device__ __forceinline__ bool update_cell(const Params &P, double lam,
                                            const CellInT<float> &c, const FluxT<float> &Fm,
                                            const FluxT<float> &Fp, double (&out)[6],
                                            bool grav = false, double hg = 0.0) {
  const bool dual = (P.flags & kDualEnergy) != 0;
  const float lf = float(lam);
  const float rn = __builtin_fmaf(-lf, Fp.m[0] - Fm.m[0], c.rho);
  float mu = __builtin_fmaf(-lf, Fp.m[1] - Fm.m[1], c.rho * c.u);
  const float m1 = __builtin_fmaf(-lf, Fp.m[2] - Fm.m[2], c.rho * c.v1);
  const float m2 = __builtin_fmaf(-lf, Fp.m[3] - Fm.m[3], c.rho * c.v2);
  const double rd = c.rho;
  double mE = rd * c.E - lam * (Fp.E - Fm.E);
  const double me = rd * c.e - lam * (double(Fp.e) - double(Fm.e)) -
                    lam * c.p * (double(Fp.ub) - double(Fm.ub));
  if (grav) {
    const float hf = float(hg);
    mu = __builtin_fmaf(hf, c.rho + rn, mu);
    mE = mE + hg * (rd * double(c.u) + double(mu));
  }
  const float irf = __builtin_amdgcn_rcpf(rn);
  const float unf = mu * irf, v1f = m1 * irf, v2f = m2 * irf;
  const double rnd = rn;
  const double ir = rcp64(rnd);
  const double un = unf, v1n = v1f, v2n = v2f;
  const double En = mE * ir, eraw = me * ir;
  const double ke = 0.5 * (un * un + v1n * v1n + v2n * v2n);
  const double epsE = En - ke;
  bool bad = !(rnd > P.rho_floor);
  double sel = epsE;
  if (dual && !ratio_above(epsE, En, P.eta1)) sel = eraw;
  if (!(sel > 0.0)) bad = true;
  double en = eraw < P.e_floor ? P.e_floor : eraw;
  if (dual && ratio_above(rnd * epsE, c.rhoEmax, P.eta2)) en = epsE;
  out[0] = rnd; out[1] = un; out[2] = v1n; out[3] = v2n; out[4] = En; out[5] = en;
  return bad;
}

// A cell still non-positive after the fallback: density raised to the floor
// (keeping the old velocity if so), pressure set to the floor.
template <class T>
__device__ __forceinline__ void floor_cell(const Params &P, const CellInT<T> &c,
                                           double (&out)[6]) {
  const double g = P.gamma;
  if (!(out[0] > P.rho_floor)) {
    out[0] = P.rho_floor;
    out[1] = double(c.u); out[2] = double(c.v1); out[3] = double(c.v2);
  }
  double eps = P.p_floor / ((g - 1.0) * out[0]);
  out[5] = eps;
  out[4] = eps + 0.5 * (out[1] * out[1] + out[2] * out[2] + out[3] * out[3]);
}

}  // namespace ppm
