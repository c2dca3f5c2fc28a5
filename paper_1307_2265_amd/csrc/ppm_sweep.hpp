// ppm_sweep.hpp -- the streaming 1-D PPM sweep of one pencil (device).
//
// One thread owns one pencil and walks it from its first to its last cell
// once.  Every quantity a later stage needs is kept in a short sliding window
// of registers, so each input cell is read from HBM once and each updated cell
// written once, with no LDS staging and no second pass.  With the head of the
// walk at cell k:
//   * cell k is loaded and its pressure and sound speed evaluated;
//   * the limited slope of cell k-1 and the interface value between k-2 and
//     k-1 are formed, and the flattening indicator of cell k-2;
//   * the parabola of cell r = k-3 is completed (steepening, flattening,
//     monotonicity) and traced to both of its edges;
//   * the Riemann problem at face (r-1)+1/2 is solved, giving the provisional
//     update of cell r-1;
//   * cell r-2 is finalised and written.  Holding the write back by one cell
//     lets the HLL fallback (Sec. "Riemann Solvers and Fallback") re-solve
//     both faces of a cell whose provisional update went non-positive and
//     redo its neighbours before anything reaches memory.  The traced states
//     the HLL solver needs are parked in LDS (one private slot pair per
//     thread) since they are read only when a fallback actually happens.
#pragma once

#include "ppm_math.hpp"

namespace ppm {

// Storage and compute types of a precision.  S: storage of rho and the
// velocity; T: reconstruction and tracing.  Energies are stored in double,
// and the pressure selection, Riemann iteration and updates run in double.
struct PrecF64 {
  using S = double;
  using T = double;
};
struct PrecMixed {
  using S = float;
  using T = float;
};

// Device copy of one patch.
struct PatchDev {
  int32_t n[3];      // active cells per axis
  int32_t ghost;
  int32_t level;
  int32_t pad;
  double dx[3];
  void *rho, *vel[3];
  double *etot, *eint;
  double *flux_reg;
  const void *acc[3];  // nullable: gravitational acceleration per axis (storage type)
};

// One pencil as the marcher sees it: fields in pencil order (normal velocity
// first), the offset of its cell 0 and the element stride along it.
template <class S> struct PencilRef {
  S *rho, *u, *v1, *v2;
  double *E, *e;
  int64_t base, stride;
  int n, g;
  double dx;
  double *reg_lo, *reg_hi;  // nullable: register slots of this pencil
  int64_t reg_stride;       // stride between the six register fields
  int lab[6];               // lab field index of each pencil-order flux slot
  const S *acc;             // nullable: acceleration along the pencil
};

// LDS of a marching thread, in doubles (strided by the block size): two
// slots of the traced L and R states of a face (for the fallback), the final
// flux of the face behind the cell about to be written (read only by the
// fallback) and that cell's provisional update, then the running CFL maximum
// of the sweeps that take one.
constexpr int kSlotDoubles = 10;
constexpr int kLdsFluxA = 2 * kSlotDoubles;
constexpr int kLdsProvA = kLdsFluxA + 7;
constexpr int kLdsMarch = kLdsProvA + 6;
constexpr int kLdsCfl = kLdsMarch;

// Lane-parallel sweep: halo lanes at each end of a 64-lane segment, cells a
// segment writes, and the pencils a wave streams in one run (about
// kStreamCells cells).
constexpr int kLaneHalo = 5;
constexpr int kLaneOut = 64 - 2 * kLaneHalo;
constexpr int kStreamCells = 32 * kLaneOut;
__host__ __device__ __forceinline__ int rows_per_wave(int n) {
  return n >= kStreamCells ? 1 : (kStreamCells + n - 1) / n;
}

// Select one of three values by a (wave-uniform) axis index without
// indexing a private array, which would live in scratch memory.
template <class V> __device__ __forceinline__ V pick3(int i, V a, V b, V c) {
  return i == 0 ? a : (i == 1 ? b : c);
}

// Offset of the block of face (2*axis + hi) in a patch's flux register.
__device__ __forceinline__ int64_t reg_face_offset(int64_t nx, int64_t ny, int64_t nz, int axis,
                                                   int hi) {
  const int64_t ax = ny * nz, ay = nx * nz, az = nx * ny;
  const int64_t before = axis == 0 ? 0 : (axis == 1 ? 2 * ax : 2 * (ax + ay));
  return 6 * (before + (hi ? pick3<int64_t>(axis, ax, ay, az) : 0));
}

// The pencil (i1, i2) of a sweep along `axis` of one patch.
template <class S>
__device__ __forceinline__ PencilRef<S> make_pencil(const PatchDev &pd, int axis, int i1, int i2) {
  const int t1 = axis == 0 ? 1 : 0, t2 = axis == 2 ? 1 : 2;
  const int g = pd.ghost;
  const int N0 = pd.n[0], N1 = pd.n[1], N2 = pd.n[2];
  const int nf0 = N0 + 2 * g, nf1 = N1 + 2 * g;
  const int Na = pick3(axis, N0, N1, N2), Nt1 = pick3(t1, N0, N1, N2), Nt2 = pick3(t2, N0, N1, N2);
  const int64_t sx = 1, sy = nf0, sz = int64_t(nf0) * nf1;
  PencilRef<S> pc;
  pc.rho = static_cast<S *>(pd.rho);
  pc.u = static_cast<S *>(pick3(axis, pd.vel[0], pd.vel[1], pd.vel[2]));
  pc.v1 = static_cast<S *>(pick3(t1, pd.vel[0], pd.vel[1], pd.vel[2]));
  pc.v2 = static_cast<S *>(pick3(t2, pd.vel[0], pd.vel[1], pd.vel[2]));
  pc.E = pd.etot;
  pc.e = pd.eint;
  pc.base = i1 * pick3(t1, sx, sy, sz) + i2 * pick3(t2, sx, sy, sz);
  pc.stride = pick3(axis, sx, sy, sz);
  pc.n = Na + 2 * g;
  pc.g = g;
  pc.dx = pick3(axis, pd.dx[0], pd.dx[1], pd.dx[2]);
  pc.reg_lo = pc.reg_hi = nullptr;
  pc.reg_stride = 0;
  pc.lab[0] = 0; pc.lab[1] = 1 + axis; pc.lab[2] = 1 + t1; pc.lab[3] = 1 + t2;
  pc.lab[4] = 4; pc.lab[5] = 5;
  pc.acc = static_cast<const S *>(pick3(axis, pd.acc[0], pd.acc[1], pd.acc[2]));
  if (pd.flux_reg && i1 >= g && i1 < g + Nt1 && i2 >= g && i2 < g + Nt2) {
    const int64_t ro = int64_t(i2 - g) * Nt1 + (i1 - g);
    pc.reg_lo = pd.flux_reg + reg_face_offset(N0, N1, N2, axis, 0) + ro;
    pc.reg_hi = pd.flux_reg + reg_face_offset(N0, N1, N2, axis, 1) + ro;
    pc.reg_stride = int64_t(Nt1) * Nt2;
  }
  return pc;
}

// Number of pencils of a sweep along `axis` of one patch: transverse axes
// restricted to their active range where `mask` says so.
__device__ __forceinline__ int pencil_count(const PatchDev &pd, int axis, int mask) {
  const int t1 = axis == 0 ? 1 : 0, t2 = axis == 2 ? 1 : 2;
  const int g = pd.ghost;
  const int Nt1 = pick3(t1, pd.n[0], pd.n[1], pd.n[2]);
  const int Nt2 = pick3(t2, pd.n[0], pd.n[1], pd.n[2]);
  const int w1 = ((mask >> t1) & 1) ? Nt1 : Nt1 + 2 * g;
  const int w2 = ((mask >> t2) & 1) ? Nt2 : Nt2 + 2 * g;
  return w1 * w2;
}

// Pencil `idx` of the sweep's pencil set in one patch: transverse axes
// restricted to their active range where `mask` says so.  False if idx is
// past the end.
__device__ __forceinline__ bool pencil_index(const PatchDev &pd, int axis, int mask, int idx,
                                             int &i1, int &i2) {
  const int t1 = axis == 0 ? 1 : 0, t2 = axis == 2 ? 1 : 2;
  const int g = pd.ghost;
  const int Nt1 = pick3(t1, pd.n[0], pd.n[1], pd.n[2]);
  const int Nt2 = pick3(t2, pd.n[0], pd.n[1], pd.n[2]);
  const bool r1 = (mask >> t1) & 1, r2 = (mask >> t2) & 1;
  const int lo1 = r1 ? g : 0, w1 = r1 ? Nt1 : Nt1 + 2 * g;
  const int lo2 = r2 ? g : 0, w2 = r2 ? Nt2 : Nt2 + 2 * g;
  if (idx >= w1 * w2) return false;
  i1 = lo1 + idx % w1;
  i2 = lo2 + idx / w1;
  return true;
}

// Hydro CFL signal speed of one cell (Sec. "Timestepping", the harmonic
// multi-D form): sum over the axes of (c_s + |v_d|) / dx_d, with c_s from the
// dual-energy pressure.  Takes the cell as stored (rho and the velocity in
// storage precision) and its velocity in pencil order (u along `axis`, then
// the two transverse components), and evaluates everything in lab axis order,
// so the CFL reduction and the last sweep of a step that accumulates the next
// step's timestep give the same value bit for bit.
template <class S>
__device__ __forceinline__ double cell_signal(const Params &P, int axis, const double (&dx)[3],
                                              S r, S u, S v1, S v2, double E, double e) {
  const double uu = double(u), a = double(v1), b = double(v2);
  const double vx = axis == 0 ? uu : a;
  const double vy = axis == 1 ? uu : (axis == 0 ? a : b);
  const double vz = axis == 2 ? uu : b;
  double p, c;
  eos(P, double(r), vx, vy, vz, E, e, p, c);
  return ddiv(c + fabs(vx), dx[0]) + ddiv(c + fabs(vy), dx[1]) + ddiv(c + fabs(vz), dx[2]);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Maximum signal speed over the cells a sweep writes, for a sweep that also
// yields the next step's timestep.  The marching sweep keeps each thread's
// running maximum in LDS (`lds`, one double per thread) to spare its vector
// registers; the lane-parallel sweep keeps each lane's in `smax`, and the
// wave maximum is taken once, when the kernel commits it.
struct CflAcc {
  int axis;
  double dx[3];
  double smax;
  double *lds;
};

__device__ __forceinline__ CflAcc cfl_acc(const PatchDev &pd, int axis, double *lds) {
  return CflAcc{axis, {pd.dx[0], pd.dx[1], pd.dx[2]}, 0.0, lds};
}

// The part of a pencil that one thread marches when two threads share a
// pencil.  The head walks cells begin .. last; the rules of the pencil's
// start (stages that need more cells than have been read yet are skipped,
// the flattening indicator of the first cells is zero, the first g cells are
// treated as ghosts) apply relative to `begin`, those of its end to the real
// end.  A thread that starts inside the pencil thereby computes its first
// cells differently from the whole march, but no cell it writes depends on
// them: a cell's update reaches five cells either side (the flattening of its
// neighbours' parabolas three, the HLL fallback of a neighbouring face two
// more), and `own_lo` is at least begin + 5 (and begin + g).  Cells own_lo ..
// own_hi are written (the faces between them, and below own_lo when own_lo is
// the pencil's first active cell, are counted); cells defer_lo .. defer_lo +
// kDeferCells - 1 go to `defer` (6 doubles per cell) instead, for the caller
// to store after the march: the other thread of the pencil reads them as
// input late in its own march.
constexpr int kDeferCells = 5;
struct MarchSpan {
  int begin, last, own_lo, own_hi, defer_lo;
  double *defer;
};

// One thread marches one pencil (or the part of it `span` gives).  kCFL: also
// take the signal speed of every cell written (the sweep must then be the
// last of its step).
// a: the level's expansion factor (1 for the static equations).  kGrav: the
// general build, with the gravity source terms (applied where the pencil has
// an acceleration field) and the optional diffusive flux.
template <class Prec, bool kCFL, bool kUseHLLC, bool kGrav>
__device__ void march_pencil(const Params &P, const PencilRef<typename Prec::S> &pc, double dt,
                             double a, double *lds_slots, int slot_stride, uint32_t &n_fallback,
                             uint32_t &n_floor, CflAcc &cfl, const MarchSpan *span = nullptr) {
  using S = typename Prec::S;
  using T = typename Prec::T;
  // with T = double the window already holds the exact pressure
  constexpr bool kExactP = sizeof(T) == sizeof(double);
  const int n = pc.n, g = pc.g;
  const int a0 = g, a1 = n - g - 1;
  // the march's own start (cell begin is its first, begin + g its first
  // active cell) and what it writes
  const bool spanned = span != nullptr;  // known where the call is inlined
  const int begin = spanned ? span->begin : 0;
  const int kend = spanned ? span->last : n - g + 4;  // the iteration that finalises its last cell
  const int b0 = begin + g;
  const int own_lo = spanned ? span->own_lo : a0, own_hi = spanned ? span->own_hi : a1;
  const int face_lo = own_lo == a0 ? a0 - 1 : own_lo;
  const bool deferring = spanned && span->defer != nullptr;
  const int defer_lo = deferring ? span->defer_lo : 0;
  auto owned = [&](int c) { return !spanned || (c >= own_lo && c <= own_hi); };
  const double lam = dt / (a * pc.dx);
  const T tlam = T(lam);
  const bool grav = kGrav && pc.acc != nullptr;
  const double hgdt = 0.5 * dt / a;
  const bool diffuse = kGrav && (P.flags & kDiffusion) != 0;
  // the diffusive flux of the face between cells jl and jl+1 (their stored
  // sweep-input values, still in memory: a cell is written two iterations
  // after its right face is final)
  auto diffuse_face = [&](FluxT<T> &F, int jl) {
    const int64_t ol = pc.base + int64_t(jl) * pc.stride, orr = ol + pc.stride;
    add_diffusion(F, double(pc.rho[ol]), double(pc.u[ol]), double(pc.v1[ol]), double(pc.v2[ol]),
                  pc.E[ol], pc.e[ol], double(pc.rho[orr]), double(pc.u[orr]),
                  double(pc.v1[orr]), double(pc.v2[orr]), pc.E[orr], pc.e[orr]);
  };
  const double gam = P.gamma;
  const bool steepen = (P.flags & kSteepen) != 0;
  const bool flatten = (P.flags & kFlatten) != 0;
  const bool fallback = (P.flags & kFallbackHLL) != 0;
  const T rho_floor = T(P.rho_floor), p_floor = T(P.p_floor);

  // Sliding windows; index 0 is the oldest cell.
  T q[5][5];       // cells k-4..k: rho, u, v1, v2, p
  double pd[5];    // cells k-4..k: pressure in double (update source term)
  T cw[2];         // cells k-3 and k-2: sound speed (cw[0] is cell r)
  T c_head;        // sound speed of the head cell
  T c_km1;
  double rE[3];    // cells k-2..k: rho*E of the sweep input
  double m3[5];    // cells k-5..k-1: max of rho*E over the cell and its neighbours
  T dm[4][5];      // cells k-4..k-1: limited slopes
  T d2[4];         // cells k-4..k-1: density second differences
  T ft[3];         // cells k-4..k-2: flattening indicators
  T fc[3][5];      // faces (k-4)+1/2 .. (k-2)+1/2: interface values
  State<T> lcarry; // left state of face r+1/2 from the previous iteration
  FluxT<T> ft_b;   // two-shock flux at face (r-2)+1/2
  // final flux at face (r-3)+1/2 and provisional update of cell A = r-2 live
  // in LDS (written every step; the flux is read only by the fallback)
  double *ff_a = lds_slots + kLdsFluxA * slot_stride;
  double *prov_a = lds_slots + kLdsProvA * slot_stride;
  bool hll_a = false;
  bool bad_a = false;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
#pragma unroll
    for (int j = 0; j < 5; ++j) q[i][j] = T(0);
    pd[i] = 0.0;
    m3[i] = 0.0;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 5; ++j) dm[i][j] = T(0);
    d2[i] = T(0);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    ft[i] = T(0);
    rE[i] = 0.0;
#pragma unroll
    for (int j = 0; j < 5; ++j) fc[i][j] = T(0);
  }
  cw[0] = cw[1] = T(0);
  c_head = c_km1 = T(0);
  lcarry = State<T>{T(0), T(0), T(0), T(0), T(0)};
  ft_b = zero_flux<T>();
#pragma unroll
  for (int j = 0; j < 7; ++j) ff_a[j * slot_stride] = 0.0;
#pragma unroll
  for (int j = 0; j < 6; ++j) prov_a[j * slot_stride] = 0.0;

  // prefetch of the head cell
  S nr = S(0), nu = S(0), nv1 = S(0), nv2 = S(0);
  double nE = 0.0, ne = 0.0;
  if (begin < n) {
    const int64_t o = pc.base + int64_t(begin) * pc.stride;
    nr = pc.rho[o]; nu = pc.u[o]; nv1 = pc.v1[o]; nv2 = pc.v2[o]; nE = pc.E[o]; ne = pc.e[o];
  }

  for (int k = begin; k <= kend; ++k) {
    const int t = k - begin;  // cells read so far, less one
    // energies of cell B = k-4 (updated below), fetched early to hide latency
    double EB = 0.0, eB = 0.0, gB = 0.0;
    if (k - 4 >= b0 && k - 4 <= a1) {
      const int64_t o = pc.base + int64_t(k - 4) * pc.stride;
      EB = pc.E[o];
      eB = pc.e[o];
      if (grav) gB = double(pc.acc[o]);
    }
    // ---- 1. head cell: load and equation of state
    if (k < n) {
      const double r = double(nr), u = double(nu), v1 = double(nv1), v2 = double(nv2);
      const double E = nE, e = ne;
      if (k + 1 < n && (!spanned || k + 1 <= kend)) {
        const int64_t o = pc.base + int64_t(k + 1) * pc.stride;
        nr = pc.rho[o]; nu = pc.u[o]; nv1 = pc.v1[o]; nv2 = pc.v2[o]; nE = pc.E[o]; ne = pc.e[o];
      }
      double p;
      T c;
      eos_cell<T>(P, r, u, v1, v2, E, e, p, c);
      q[4][0] = T(r); q[4][1] = T(u); q[4][2] = T(v1); q[4][3] = T(v2); q[4][4] = T(p);
      if (!kExactP) pd[4] = p;
      c_head = c;
      rE[2] = r * E;
    }
    // ---- 2. slope and second difference of cell k-1, max rho*E around it
    if (t >= 2 && k <= n - 1) {
#pragma unroll
      for (int j = 0; j < 5; ++j) dm[3][j] = limited_slope<T>(q[2][j], q[3][j], q[4][j]);
      d2[3] = second_diff<T>(q[2][0], q[3][0], q[4][0]);
      m3[4] = vmax<double>(vmax<double>(rE[0], rE[1]), rE[2]);
    }
    // ---- 3. interface value between cells k-2 and k-1
    if (t >= 3 && k <= n - 1) {
#pragma unroll
      for (int j = 0; j < 5; ++j) fc[2][j] = interface_value<T>(q[2][j], q[3][j], dm[2][j], dm[3][j]);
    }
    // ---- 4. flattening indicator of cell k-2 (zero where its stencil leaves the pencil)
    ft[2] = T(0);
    if (flatten && t >= 4 && k <= n - 1)
      ft[2] = flatten_indicator<T>(q[0][4], q[1][4], q[3][4], q[4][4], q[1][1], q[3][1]);

    // ---- 5. parabola of cell r = k-3, traced to both edges
    const int r = k - 3;
    State<T> rstate = lcarry, lnew = lcarry;
    const bool need_left_edge = r >= b0 && r <= a1 + 1;   // right state of face (r-1)+1/2
    const bool need_right_edge = r >= b0 - 1 && r <= a1;  // left state of face r+1/2
    if (need_left_edge || need_right_edge) {
      T l[5], rr[5], dq[5], q6[5];
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        l[j] = fc[0][j];   // face (r-1)+1/2
        rr[j] = fc[1][j];  // face r+1/2
      }
      if (steepen) {
        T eta = steepen_eta<T>(gam, q[0][0], q[2][0], q[0][4], q[2][4], d2[0], d2[2]);
        if (eta != T(0)) {
          l[0] = mad<T>(l[0], T(1) - eta, mad<T>(T(0.5), dm[0][0], q[0][0]) * eta);
          rr[0] = mad<T>(rr[0], T(1) - eta, mad<T>(T(-0.5), dm[2][0], q[2][0]) * eta);
        }
      }
      if (flatten) {
        T fn = (q[2][4] - q[0][4] > T(0)) ? ft[0] : ft[2];
        T f = vmax<T>(ft[1], fn);
        if (f != T(0)) {
#pragma unroll
          for (int j = 0; j < 5; ++j) {
            l[j] = mad<T>(f, q[1][j], (T(1) - f) * l[j]);
            rr[j] = mad<T>(f, q[1][j], (T(1) - f) * rr[j]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 5; ++j) monotonize<T>(q[1][j], l[j], rr[j], dq[j], q6[j]);
      const T u = q[1][1], c = cw[0];
      if (need_left_edge)
        rstate = trace_edge<T, false>(gam, l, rr, dq, q6, u, c, tlam, rho_floor, p_floor);
      if (need_right_edge)
        lnew = trace_edge<T, true>(gam, l, rr, dq, q6, u, c, tlam, rho_floor, p_floor);
    }

    // ---- 6. Riemann problem at face fc = (r-1)+1/2
    FluxT<T> ft_c = zero_flux<T>();
    double *slot_c = lds_slots + (k & 1) * kSlotDoubles * slot_stride;
    if (r - 1 >= b0 - 1 && r - 1 <= a1) {
      ft_c = face_flux<kUseHLLC, T>(P, lcarry, rstate);
      if (diffuse) diffuse_face(ft_c, r - 1);
      if (fallback) {
        slot_c[0 * slot_stride] = double(lcarry.r);
        slot_c[1 * slot_stride] = double(lcarry.u);
        slot_c[2 * slot_stride] = double(lcarry.v1);
        slot_c[3 * slot_stride] = double(lcarry.v2);
        slot_c[4 * slot_stride] = double(lcarry.p);
        slot_c[5 * slot_stride] = double(rstate.r);
        slot_c[6 * slot_stride] = double(rstate.u);
        slot_c[7 * slot_stride] = double(rstate.v1);
        slot_c[8 * slot_stride] = double(rstate.v2);
        slot_c[9 * slot_stride] = double(rstate.p);
      }
    }

    // ---- 7. provisional update of cell B = r-1 with the two-shock fluxes
    const int B = r - 1;
    bool bad_b = false;
    double prov_b[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (B >= b0 && B <= a1) {
      CellInT<T> cin;
      cin.rho = q[0][0]; cin.u = q[0][1];
      cin.v1 = q[0][2]; cin.v2 = q[0][3];
      cin.E = EB; cin.e = eB;
      cin.p = kExactP ? double(q[0][4]) : pd[0];
      cin.rhoEmax = m3[1];
      bad_b = update_cell(P, lam, cin, ft_b, ft_c, prov_b, grav, hgdt * gB);
    }

    // ---- 8. face fb = (r-2)+1/2 becomes final: HLL if a neighbour went bad
    const int A = r - 2;
    const int fb = r - 2;  // face index: fb+1/2 lies between cells A and B
    FluxT<T> ff_b = ft_b;
    bool hll_b = false;
    if (fb >= b0 - 1 && fb <= a1) {
      hll_b = fallback && (bad_a || bad_b);
      if (hll_b) {
        const double *slot_b = lds_slots + ((k - 1) & 1) * kSlotDoubles * slot_stride;
        double sl[5], sr[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          sl[j] = slot_b[j * slot_stride];
          sr[j] = slot_b[(5 + j) * slot_stride];
        }
        ff_b = narrow_flux<T>(hll_flux(P, sl, sr));
        if (diffuse) diffuse_face(ff_b, fb);
        if (!spanned || (fb >= face_lo && fb <= own_hi)) ++n_fallback;
      }
      if (fb == a0 - 1 && pc.reg_lo) {
#pragma unroll
        for (int j = 0; j < 6; ++j) pc.reg_lo[pc.lab[j] * pc.reg_stride] = dt * ff_b.get(j);
      }
      if (fb == a1 && pc.reg_hi) {
#pragma unroll
        for (int j = 0; j < 6; ++j) pc.reg_hi[pc.lab[j] * pc.reg_stride] = dt * ff_b.get(j);
      }
    }

    // ---- 9. finalise and write cell A = r-2
    if (A >= b0 && A <= a1) {
      const int64_t o = pc.base + int64_t(A) * pc.stride;
      double out[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) out[j] = prov_a[j * slot_stride];
      bool bad = bad_a;
      if (hll_a || hll_b) {
        // redo the update with the final fluxes (input of A is still in memory)
        CellInT<T> cin;
        cin.rho = T(pc.rho[o]); cin.u = T(pc.u[o]);
        cin.v1 = T(pc.v1[o]); cin.v2 = T(pc.v2[o]);
        cin.E = pc.E[o]; cin.e = pc.e[o];
        double pp, cc;
        eos(P, double(cin.rho), double(cin.u), double(cin.v1), double(cin.v2), cin.E, cin.e, pp,
            cc);
        cin.p = pp;
        cin.rhoEmax = m3[0];
        FluxT<T> fa;
#pragma unroll
        for (int j = 0; j < 7; ++j) fa.set(j, ff_a[j * slot_stride]);
        bad = update_cell(P, lam, cin, fa, ff_b, out, grav,
                          grav ? hgdt * double(pc.acc[o]) : 0.0);
      }
      if (bad) {
        CellInT<T> cin;
        cin.rho = T(pc.rho[o]); cin.u = T(pc.u[o]);
        cin.v1 = T(pc.v1[o]); cin.v2 = T(pc.v2[o]);
        cin.E = pc.E[o]; cin.e = pc.e[o]; cin.p = 0.0; cin.rhoEmax = 0.0;
        floor_cell(P, cin, out);
        if (owned(A)) ++n_floor;
      }
      if (owned(A)) {
        if (deferring && A >= defer_lo && A < defer_lo + kDeferCells) {
          double *d = span->defer + (A - defer_lo) * 6;
#pragma unroll
          for (int j = 0; j < 4; ++j) d[j] = double(S(out[j]));
          d[4] = out[4];
          d[5] = out[5];
        } else {
          pc.rho[o] = S(out[0]);
          pc.u[o] = S(out[1]);
          pc.v1[o] = S(out[2]);
          pc.v2[o] = S(out[3]);
          pc.E[o] = out[4];
          pc.e[o] = out[5];
        }
        if (kCFL) {
          const double s = cell_signal<S>(P, cfl.axis, cfl.dx, S(out[0]), S(out[1]), S(out[2]),
                                          S(out[3]), out[4], out[5]);
          const double m = *cfl.lds;
          *cfl.lds = s > m ? s : m;
        }
      }
    }

    // ---- 10. carry the face and cell state one step
#pragma unroll
    for (int j = 0; j < 7; ++j) ff_a[j * slot_stride] = ff_b.get(j);
    hll_a = hll_b;
    ft_b = ft_c;
#pragma unroll
    for (int j = 0; j < 6; ++j) prov_a[j * slot_stride] = prov_b[j];
    bad_a = bad_b;
    lcarry = lnew;

    // ---- 11. shift the windows
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int j = 0; j < 5; ++j) q[i][j] = q[i + 1][j];
      if (!kExactP) pd[i] = pd[i + 1];
      m3[i] = m3[i + 1];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int j = 0; j < 5; ++j) dm[i][j] = dm[i + 1][j];
      d2[i] = d2[i + 1];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ft[i] = ft[i + 1];
      rE[i] = rE[i + 1];
#pragma unroll
      for (int j = 0; j < 5; ++j) fc[i][j] = fc[i + 1][j];
    }
    cw[0] = cw[1];
    cw[1] = c_km1;
    c_km1 = c_head;
  }
}

}  // namespace ppm
