// exact_riemann.cpp -- TEST INFRASTRUCTURE ONLY.
//
// Exact solution of the Riemann problem for the 1-D Euler equations of an
// ideal gas, used to pin the oracle's two-shock solver (exact whenever both
// waves are shocks) and its full sweeps (Sod's shock tube, Sec. "Sod Shock
// Tube").  Textbook construction (Toro 1997, ch. 4, which the paper cites for
// its Riemann solvers): the star pressure is the root of
//   f(p) = f_L(p) + f_R(p) + (u_R - u_L),
// where f_K is the velocity change across a shock (Rankine-Hugoniot) when
// p > p_K and across a rarefaction (isentropic, Riemann invariant) when
// p <= p_K.  The root is bracketed and bisected to the last bit, then the
// self-similar solution is sampled at x/t = xi.

#include <cmath>

#include "ppm_oracle.h"

namespace {

struct Side {
  double rho, u, p, c;
};

// Velocity change across the left or right wave when the star pressure is p.
double fK(double p, const Side &s, double g) {
  if (p > s.p) {
    double A = 2.0 / ((g + 1.0) * s.rho);
    double B = (g - 1.0) / (g + 1.0) * s.p;
    return (p - s.p) * std::sqrt(A / (p + B));
  }
  return 2.0 * s.c / (g - 1.0) * (std::pow(p / s.p, (g - 1.0) / (2.0 * g)) - 1.0);
}

double star_pressure(const Side &L, const Side &R, double g) {
  auto f = [&](double p) { return fK(p, L, g) + fK(p, R, g) + (R.u - L.u); };
  double lo = 0.0, hi = L.p > R.p ? L.p : R.p;
  if (f(lo) >= 0.0) return 0.0;  // the waves leave a vacuum
  while (f(hi) < 0.0) hi *= 2.0;
  for (int it = 0; it < 400; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (f(mid) < 0.0) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// Star-region density next to side s.
double star_density(double ps, const Side &s, double g) {
  if (ps > s.p) {
    double r = ps / s.p, k = (g - 1.0) / (g + 1.0);
    return s.rho * (r + k) / (k * r + 1.0);
  }
  return s.rho * std::pow(ps / s.p, 1.0 / g);
}

void sample(double xi, const Side &L, const Side &R, double ps, double us, double g,
            double *rho, double *u, double *p) {
  const double gm = (g - 1.0) / (2.0 * g), gp = (g + 1.0) / (2.0 * g);
  if (xi <= us) {  // left of the contact
    if (ps > L.p) {
      double S = L.u - L.c * std::sqrt(gp * ps / L.p + gm);
      if (xi <= S) { *rho = L.rho; *u = L.u; *p = L.p; }
      else { *rho = star_density(ps, L, g); *u = us; *p = ps; }
    } else {
      double head = L.u - L.c;
      double cs = L.c * std::pow(ps / L.p, gm);
      double tail = us - cs;
      if (xi <= head) { *rho = L.rho; *u = L.u; *p = L.p; }
      else if (xi > tail) { *rho = star_density(ps, L, g); *u = us; *p = ps; }
      else {
        double b = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * L.c) * (L.u - xi);
        *rho = L.rho * std::pow(b, 2.0 / (g - 1.0));
        *u = 2.0 / (g + 1.0) * (L.c + 0.5 * (g - 1.0) * L.u + xi);
        *p = L.p * std::pow(b, 2.0 * g / (g - 1.0));
      }
    }
  } else {  // right of the contact
    if (ps > R.p) {
      double S = R.u + R.c * std::sqrt(gp * ps / R.p + gm);
      if (xi >= S) { *rho = R.rho; *u = R.u; *p = R.p; }
      else { *rho = star_density(ps, R, g); *u = us; *p = ps; }
    } else {
      double head = R.u + R.c;
      double cs = R.c * std::pow(ps / R.p, gm);
      double tail = us + cs;
      if (xi >= head) { *rho = R.rho; *u = R.u; *p = R.p; }
      else if (xi < tail) { *rho = star_density(ps, R, g); *u = us; *p = ps; }
      else {
        double b = 2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * R.c) * (R.u - xi);
        *rho = R.rho * std::pow(b, 2.0 / (g - 1.0));
        *u = 2.0 / (g + 1.0) * (-R.c + 0.5 * (g - 1.0) * R.u + xi);
        *p = R.p * std::pow(b, 2.0 * g / (g - 1.0));
      }
    }
  }
}

}  // namespace

extern "C" void ppmo_exact_riemann(double g, const double l[3], const double r[3], int32_t nxi,
                                   const double *xi, double *rho, double *u, double *p,
                                   double star[4]) {
  Side L = {l[0], l[1], l[2], std::sqrt(g * l[2] / l[0])};
  Side R = {r[0], r[1], r[2], std::sqrt(g * r[2] / r[0])};
  double ps = star_pressure(L, R, g);
  double us = 0.5 * (L.u + R.u) + 0.5 * (fK(ps, R, g) - fK(ps, L, g));
  if (star) {
    star[0] = ps; star[1] = us;
    star[2] = star_density(ps, L, g); star[3] = star_density(ps, R, g);
  }
  for (int k = 0; k < nxi; ++k) sample(xi[k], L, R, ps, us, g, &rho[k], &u[k], &p[k]);
}
