// ppm_lanes.hpp -- the 1-D PPM sweep with the cells of a pencil across the
// lanes of a wave (device).
//
// A wavefront streams a run of consecutive pencils (rows) of one patch,
// concatenated, through segments of 64 consecutive cells, so every load and
// store of a sweep along x is one coalesced access per field, and every stage
// of the update is evaluated for 64 cells at once, reading its neighbours'
// values from the adjacent lanes with cross-lane shuffles.  The update of a
// cell depends on the five cells either side of it in its own pencil (the
// flattening of its neighbours' parabolas reaches three cells out, the HLL
// fallback of a neighbouring face two more), so a segment writes its 54
// middle cells and the 5 lanes at each end only supply halo values.
// Segments overlap by 10 cells; since the pencils are updated in place, the
// next segment takes those cells' inputs from the registers of the previous
// one (a lane permute) rather than from memory, where some were already
// overwritten.  Where a segment spans the end of one pencil and the start of
// the next, a lane reads its neighbour pencil's cell where the sweep would
// read a cell outside its own pencil; every stage tests the position of its
// cell within its pencil against the same ranges the pencil-marching sweep
// uses, so no valid result uses such a value and both sweeps give the same
// result bit for bit.  Streaming many short pencils back to back keeps 54 of
// 64 lanes productive whatever the pencil length.
#pragma once

#include "ppm_sweep.hpp"

namespace ppm {


// Neighbour values by whole-wave DPP shifts (one VALU move per 32 bits, no
// LDS round trip): wave_shr:1 gives lane i the value of lane i-1, wave_shl:1
// that of lane i+1; the lane with no source (0, resp. 63) reads zero, which
// needs no copy of an old value into the destination first.  Lanes 0 and 63
// are halo lanes, whose results no written cell uses; the Riemann solve,
// whose iteration a zero state would drive to its cap, is confined to the
// lanes whose face can reach a written cell (need_face below).
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;

template <int kCtrl> __device__ __forceinline__ int dpp_shift32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, kCtrl, 0xf, 0xf, true);
}

template <int kCtrl, class V> __device__ __forceinline__ V dpp_shift(V v) {
  static_assert(sizeof(V) == 4 || sizeof(V) == 8, "32- or 64-bit values");
  if constexpr (sizeof(V) == 8) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = unsigned(dpp_shift32<kCtrl>(int(unsigned(b))));
    const unsigned hi = unsigned(dpp_shift32<kCtrl>(int(unsigned(b >> 32))));
    return __builtin_bit_cast(V, (unsigned long long)hi << 32 | lo);
  } else {
    return __builtin_bit_cast(V, dpp_shift32<kCtrl>(__builtin_bit_cast(int, v)));
  }
}

template <class V> __device__ __forceinline__ V from_left(V v) { return dpp_shift<kDppWaveShr1>(v); }
template <class V> __device__ __forceinline__ V from_right(V v) { return dpp_shift<kDppWaveShl1>(v); }
template <class V> __device__ __forceinline__ V from_left2(V v) { return from_left(from_left(v)); }
template <class V> __device__ __forceinline__ V from_right2(V v) { return from_right(from_right(v)); }

template <class T> __device__ __forceinline__ FluxT<T> flux_from_left(const FluxT<T> &F) {
  FluxT<T> o;
#pragma unroll
  for (int k = 0; k < 4; ++k) o.m[k] = from_left(F.m[k]);
  o.E = from_left(F.E);
  o.e = from_left(F.e);
  o.ub = from_left(F.ub);
  return o;
}

template <class T> __device__ __forceinline__ State<T> state_from_right(const State<T> &s) {
  return State<T>{from_right(s.r), from_right(s.u), from_right(s.v1), from_right(s.v2),
                  from_right(s.p)};
}

// Input of one cell as loaded (rho and velocities promoted to double).
struct CellLoad {
  double r, u, v1, v2, E, e;
};

// One segment: lane holds cell j of pencil pc (j = -1 for a placeholder
// lane beyond the stream, which no valid result uses).  `in` is this lane's
// input cell; the lane writes its cell (and counts its events) if `mine`,
// and solves the Riemann problem of its face j+1/2 only if `need_face` (the
// face's provisional flux can reach a written cell or the face the caller
// reads).
// lam = dt / (a pc.dx) and hgdt = (dt / 2) / a, with a the level's expansion
// factor (the same for every pencil of the patch).  Returns the final flux
// (after the fallback) of face j+1/2.
template <class Prec, bool kCFL, bool kUseHLLC, bool kGrav>
__device__ FluxT<typename Prec::T> sweep_segment(const Params &P, const PencilRef<typename Prec::S> &pc, double dt,
                              double lam, double hgdt, int j, bool mine, bool need_face,
                              const CellLoad &in, uint32_t &n_fallback, uint32_t &n_floor,
                              CflAcc &cfl) {
  using S = typename Prec::S;
  using T = typename Prec::T;
  const int n = pc.n, g = pc.g;
  const int a0 = g, a1 = n - g - 1;
  const T tlam = T(lam);
  const double gam = P.gamma;
  const bool steepen = (P.flags & kSteepen) != 0;
  const bool flatten = (P.flags & kFlatten) != 0;
  const bool fallback = (P.flags & kFallbackHLL) != 0;

  // ---- equation of state
  const bool has = j >= 0 && j < n;
  const int64_t o = pc.base + int64_t(has ? j : 0) * pc.stride;
  const double r = in.r, u = in.u, v1 = in.v1, v2 = in.v2, E = in.E, e = in.e;
  double pd;
  T cc;
  eos_cell<T>(P, r, u, v1, v2, E, e, pd, cc);
  T q[5] = {T(r), T(u), T(v1), T(v2), T(pd)};
  const double rE = r * E;

  // ---- neighbours
  T qm[5], qp[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    qm[k] = from_left(q[k]);
    qp[k] = from_right(q[k]);
  }
  const double rEm = from_left(rE), rEp = from_right(rE);
  const double m3 = vmax<double>(vmax<double>(rEm, rE), rEp);

  // ---- limited slopes (cells 1..n-2), density second difference
  T dm[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) dm[k] = limited_slope<T>(qm[k], q[k], qp[k]);
  const T d2 = second_diff<T>(qm[0], q[0], qp[0]);

  // ---- interface value at face j+1/2 (cells 1..n-3)
  T face[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) face[k] = interface_value<T>(q[k], qp[k], dm[k], from_right(dm[k]));

  // ---- flattening indicator (cells 2..n-3, else zero)
  T ft = T(0);
  if (flatten) {
    const T pm2 = from_left2(q[4]), pp2 = from_right2(q[4]);
    if (j >= 2 && j <= n - 3) ft = flatten_indicator<T>(pm2, qm[4], qp[4], pp2, qm[1], qp[1]);
  }

  // ---- parabola of cell j, traced to both edges
  T l[5], rr[5], dq[5], q6[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    l[k] = from_left(face[k]);  // face (j-1)+1/2
    rr[k] = face[k];
  }
  if (steepen) {
    const T d2m = from_left(d2), d2p = from_right(d2);
    const T dmm = from_left(dm[0]), dmp = from_right(dm[0]);
    T eta = steepen_eta<T>(gam, qm[0], qp[0], qm[4], qp[4], d2m, d2p);
    if (eta != T(0)) {
      l[0] = mad<T>(l[0], T(1) - eta, mad<T>(T(0.5), dmm, qm[0]) * eta);
      rr[0] = mad<T>(rr[0], T(1) - eta, mad<T>(T(-0.5), dmp, qp[0]) * eta);
    }
  }
  if (flatten) {
    const T ftm = from_left(ft), ftp = from_right(ft);
    T fn = (qp[4] - qm[4] > T(0)) ? ftm : ftp;
    T f = vmax<T>(ft, fn);
    if (f != T(0)) {
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        l[k] = mad<T>(f, q[k], (T(1) - f) * l[k]);
        rr[k] = mad<T>(f, q[k], (T(1) - f) * rr[k]);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) monotonize<T>(q[k], l[k], rr[k], dq[k], q6[k]);
  const T rho_floor = T(P.rho_floor), p_floor = T(P.p_floor);
  // left state of face j+1/2 (from this cell) and right state of face
  // (j-1)+1/2 (from this cell); face j+1/2 takes its right state from lane j+1
  const State<T> sl = trace_edge<T, true>(gam, l, rr, dq, q6, q[1], cc, tlam, rho_floor, p_floor);
  const State<T> srown = trace_edge<T, false>(gam, l, rr, dq, q6, q[1], cc, tlam, rho_floor, p_floor);
  const State<T> sr = state_from_right(srown);

  // ---- Riemann problem at face j+1/2 (faces a0-1..a1), with the optional
  // diffusive flux from this cell's and the right neighbour's input values
  const bool face_ok = need_face && j >= a0 - 1 && j <= a1;
  const bool diffuse = kGrav && (P.flags & kDiffusion) != 0;
  // the diffusive flux, from this cell's and the right neighbour's input
  // values (the shifts run on every lane, outside divergent branches)
  auto diffuse_into = [&](FluxT<T> &G) {
    const double nr = from_right(in.r), nu = from_right(in.u), nv1 = from_right(in.v1);
    const double nv2 = from_right(in.v2), nE = from_right(in.E), ne = from_right(in.e);
    if (face_ok) add_diffusion(G, in.r, in.u, in.v1, in.v2, in.E, in.e, nr, nu, nv1, nv2, nE, ne);
  };
  FluxT<T> F = zero_flux<T>();
  if (face_ok) F = face_flux<kUseHLLC, T>(P, sl, sr);
  if (diffuse) diffuse_into(F);

  // ---- provisional update of cell j (a0..a1)
  const bool cell_ok = j >= a0 && j <= a1;
  CellInT<T> cin;
  cin.rho = T(r); cin.u = T(u); cin.v1 = T(v1); cin.v2 = T(v2);
  cin.E = E; cin.e = e; cin.p = pd;
  cin.rhoEmax = m3;
  double out[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  FluxT<T> Fm = flux_from_left(F);
  bool bad = false;
  const bool grav = kGrav && pc.acc != nullptr;
  const double hg = grav && cell_ok ? hgdt * double(pc.acc[o]) : 0.0;
  if (cell_ok) bad = update_cell(P, lam, cin, Fm, F, out, grav, hg);
  // the lane to the right holds cell j+1 of the same pencil whenever j+1 is
  // a cell this lane's results are needed for
  const bool mine_next = from_right(int(mine)) != 0;

  // ---- HLL fallback on faces next to a non-positive cell, then redo
  if (fallback) {
    const bool bad_next = from_right(int(bad)) != 0;
    const bool hll = face_ok && (bad || bad_next);
    if (__any(hll)) {
      FluxT<T> H = F;
      if (hll) {
        const double L5[5] = {double(sl.r), double(sl.u), double(sl.v1), double(sl.v2), double(sl.p)};
        const double R5[5] = {double(sr.r), double(sr.u), double(sr.v1), double(sr.v2), double(sr.p)};
        H = narrow_flux<T>(hll_flux(P, L5, R5));
      }
      if (diffuse) diffuse_into(H);
      if (hll) {
        F = H;
        // face j+1/2 is counted by the wave that writes cell j (or cell a0 for the first face)
        if (mine || (j == a0 - 1 && mine_next)) ++n_fallback;
      }
      const bool hll_prev = from_left(int(hll)) != 0;
      Fm = flux_from_left(F);
      if (cell_ok && (hll || hll_prev)) bad = update_cell(P, lam, cin, Fm, F, out, grav, hg);
    }
  }
  if (cell_ok && bad) {
    floor_cell(P, cin, out);
    if (mine) ++n_floor;
  }

  // ---- boundary flux registers and write-back
  if (pc.reg_lo && j == a0 - 1 && mine_next) {
#pragma unroll
    for (int k = 0; k < 6; ++k) pc.reg_lo[pc.lab[k] * pc.reg_stride] = dt * F.get(k);
  }
  if (pc.reg_hi && j == a1 && mine) {
#pragma unroll
    for (int k = 0; k < 6; ++k) pc.reg_hi[pc.lab[k] * pc.reg_stride] = dt * F.get(k);
  }
  double sig = 0.0;
  if (cell_ok && mine) {
    pc.rho[o] = S(out[0]);
    pc.u[o] = S(out[1]);
    pc.v1[o] = S(out[2]);
    pc.v2[o] = S(out[3]);
    pc.E[o] = out[4];
    pc.e[o] = out[5];
    if (kCFL)
      sig = cell_signal<S>(P, cfl.axis, cfl.dx, S(out[0]), S(out[1]), S(out[2]), S(out[3]),
                           out[4], out[5]);
  }
  if (kCFL) cfl.smax = sig > cfl.smax ? sig : cfl.smax;  // per lane; reduced at the end
  return F;
}

// One wave streams pencils first .. first+nrows-1 of a sweep's pencil set,
// concatenated, segment by segment.
// a: the patch level's expansion factor.
template <class Prec, bool kCFL, bool kUseHLLC, bool kGrav>
__device__ void sweep_rows_lanes(const Params &P, const PatchDev &pd, int axis, int mask,
                                 int first, int nrows, double dt, double a, uint32_t &n_fallback,
                                 uint32_t &n_floor, CflAcc &cfl) {
  using S = typename Prec::S;
  const int lane = threadIdx.x & 63;
  const int n = (axis == 0 ? pd.n[0] : (axis == 1 ? pd.n[1] : pd.n[2])) + 2 * pd.ghost;
  const int L = nrows * n;
  const int nseg = (L + kLaneOut - 1) / kLaneOut;
  const double lam = dt / (a * pick3(axis, pd.dx[0], pd.dx[1], pd.dx[2]));
  const double hgdt = 0.5 * dt / a;
  CellLoad cur = {1.0, 0.0, 0.0, 0.0, 1.0, 1.0};
  for (int s = 0; s < nseg; ++s) {
    const int t = s * kLaneOut - kLaneHalo + lane;  // stream position of this lane
    const bool in = t >= 0 && t < L;
    const int row = in ? t / n : 0;
    const int j = in ? t - row * n : -1;
    int i1 = pd.ghost, i2 = pd.ghost;
    pencil_index(pd, axis, mask, first + row, i1, i2);
    const PencilRef<S> pc = make_pencil<S>(pd, axis, i1, i2);
    // the first 2*halo lanes overlap the previous segment's last lanes
    CellLoad prev;
    prev.r = __shfl(cur.r, lane + kLaneOut, 64);
    prev.u = __shfl(cur.u, lane + kLaneOut, 64);
    prev.v1 = __shfl(cur.v1, lane + kLaneOut, 64);
    prev.v2 = __shfl(cur.v2, lane + kLaneOut, 64);
    prev.E = __shfl(cur.E, lane + kLaneOut, 64);
    prev.e = __shfl(cur.e, lane + kLaneOut, 64);
    if (s > 0 && lane < 2 * kLaneHalo) {
      cur = prev;
    } else if (in) {
      const int64_t o = pc.base + int64_t(j) * pc.stride;
      cur.r = double(pc.rho[o]); cur.u = double(pc.u[o]);
      cur.v1 = double(pc.v1[o]); cur.v2 = double(pc.v2[o]);
      cur.E = pc.E[o]; cur.e = pc.e[o];
    } else {
      cur = CellLoad{1.0, 0.0, 0.0, 0.0, 1.0, 1.0};
    }
    const bool mine = in && lane >= kLaneHalo && lane < kLaneHalo + kLaneOut;
    // the written cells' faces, and the provisional fluxes of the faces one
    // further out that the fallback tests of the end cells read
    const bool need_face = lane >= kLaneHalo - 2 && lane <= kLaneHalo + kLaneOut;
    sweep_segment<Prec, kCFL, kUseHLLC, kGrav>(P, pc, dt, lam, hgdt, j, mine, need_face, cur,
                                               n_fallback, n_floor, cfl);
  }
}

}  // namespace ppm
