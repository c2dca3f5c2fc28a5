// ppm_api.cpp -- the C ABI declared in include/ppm.h.
//
// A plan holds a device copy of the patch table and, for every sweep axis and
// every choice of restricted transverse axes, a prefix array of pencil-chunk
// counts, so that a sweep over any set of uneven patches is one launch of a
// flat grid.  Argument validation happens here, before anything is enqueued.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <limits>
#include <sstream>
#include <string>
#include <vector>

#include "ppm.h"
#include "ppm_kernels.hpp"
#include "ppm_plan.hpp"


namespace ppm_detail {

thread_local std::string g_last_error;

ppm_status fail(ppm_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

ppm_status hip_fail(hipError_t e, const char *what) {
  return fail(PPM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// The smallest float not below x (x a positive double in the float range).
double float_at_or_above(double x) {
  float f = float(x);
  if (double(f) < x) f = std::nextafter(f, FLT_MAX);
  return double(f);
}

ppm_status check_params(const ppm_params *p) {
  if (!p) return fail(PPM_EINVAL, "params is NULL");
  if (!(p->gamma > 1.0) || !std::isfinite(p->gamma)) return fail(PPM_EINVAL, "gamma must be > 1");
  if (!(p->cfl > 0.0 && p->cfl <= 1.0)) return fail(PPM_EINVAL, "cfl must be in (0, 1]");
  if (!(p->eta1 >= 0.0) || !(p->eta2 >= 0.0)) return fail(PPM_EINVAL, "eta1/eta2 must be >= 0");
  if (!(p->rho_floor >= 1e-100) || !(p->p_floor >= 1e-100) || !(p->e_floor > 0.0))
    return fail(PPM_EINVAL, "rho_floor and p_floor must be >= 1e-100, e_floor > 0");
  if (!(p->riemann_rtol > 0.0)) return fail(PPM_EINVAL, "riemann_rtol must be > 0");
  if (p->riemann_max_iter < 1 || p->riemann_max_iter > 1000)
    return fail(PPM_EINVAL, "riemann_max_iter must be in [1, 1000]");
  if (p->flags & ~uint32_t(PPM_ALL_FLAGS | PPM_HLLC | PPM_DIFFUSION))
    return fail(PPM_EINVAL, "unknown flag bits 0x%x", p->flags);
  return PPM_OK;
}

ppm_status check_patch(const ppm_patch &q, int i, int32_t nlevels) {
  if (q.nx < 1 || q.ny < 1 || q.nz < 1)
    return fail(PPM_EINVAL, "patch %d: active dims must be >= 1", i);
  if (q.ghost < 3 || q.ghost > 6) return fail(PPM_EINVAL, "patch %d: ghost must be in 3..6", i);
  if (q.level < 0 || q.level >= nlevels)
    return fail(PPM_EINVAL, "patch %d: level %d outside [0, %d)", i, q.level, nlevels);
  if (q.bc != PPM_BC_PERIODIC && q.bc != PPM_BC_SUPPLIED)
    return fail(PPM_EINVAL, "patch %d: bc must be PPM_BC_PERIODIC or PPM_BC_SUPPLIED", i);
  if (!(q.dx > 0.0) || !(q.dy > 0.0) || !(q.dz > 0.0) || !std::isfinite(q.dx) ||
      !std::isfinite(q.dy) || !std::isfinite(q.dz))
    return fail(PPM_EINVAL, "patch %d: cell widths must be finite and > 0", i);
  if (!q.rho || !q.vx || !q.vy || !q.vz || !q.etot || !q.eint)
    return fail(PPM_EINVAL, "patch %d: NULL field pointer", i);
  if (!((q.gx && q.gy && q.gz) || (!q.gx && !q.gy && !q.gz)))
    return fail(PPM_EINVAL, "patch %d: acceleration needs all of gx, gy, gz or none", i);
  const int64_t lim = int64_t(1) << 30;
  const int64_t nf[3] = {int64_t(q.nx) + 2 * q.ghost, int64_t(q.ny) + 2 * q.ghost,
                         int64_t(q.nz) + 2 * q.ghost};
  if (nf[0] > lim || nf[1] > lim || nf[2] > lim || nf[0] * nf[1] > lim)
    return fail(PPM_EINVAL, "patch %d: too large (a face of the ghosted box exceeds 2^30 cells)", i);
  return PPM_OK;
}

ppm_status check_mixed_floors(ppm_precision prec, const ppm_params *p) {
  // PPM_MIXED stores the density in float: a floor must be a normal float
  if (prec == PPM_MIXED &&
      (!(p->rho_floor >= double(FLT_MIN)) || !(p->rho_floor <= double(FLT_MAX)) ||
       !(p->p_floor >= double(FLT_MIN)) || !(p->p_floor <= double(FLT_MAX))))
    return fail(PPM_EINVAL,
                "PPM_MIXED: rho_floor and p_floor must lie in the normal float range [%g, %g]",
                double(FLT_MIN), double(FLT_MAX));
  return PPM_OK;
}

ppm::Params device_params(ppm_precision prec, const ppm_params *p) {
  ppm::Params P;
  std::memcpy(&P, p, sizeof(ppm_params));
  static_assert(offsetof(ppm::Params, expand) == sizeof(ppm_params), "params layout");
  P.expand = nullptr;
  P.shock_k0 = std::sqrt((p->gamma - 1.0) / (2.0 * p->gamma));
  if (prec == PPM_MIXED) {  // floors a float density and pressure can hold exactly
    P.rho_floor = float_at_or_above(p->rho_floor);
    P.p_floor = float_at_or_above(p->p_floor);
  }
  return P;
}

}  // namespace ppm_detail

using ppm_detail::fail;
using ppm_detail::hip_fail;

namespace {

const int kOrders[6][3] = {{0, 1, 2}, {2, 1, 0}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}};
using ppm_detail::check_params;
using ppm_detail::check_patch;
using ppm_detail::float_at_or_above;
// Largest patch (active cells) that one workgroup of the persistent launch owns.
const int64_t kPersistentMaxCells = int64_t(1) << 21;

inline int t1_of(int axis) { return axis == 0 ? 1 : 0; }
inline int t2_of(int axis) { return axis == 2 ? 1 : 2; }
inline int tmask_of(int axis, int mask) {
  return ((mask >> t1_of(axis)) & 1) | (((mask >> t2_of(axis)) & 1) << 1);
}

ppm_status parse_tiles(ppm_plan *pl, const char *cfg) {
  if (!cfg) return PPM_OK;
  std::istringstream ss(cfg);
  std::string tok;
  while (ss >> tok) {
    const size_t eq = tok.find('=');
    if (eq == std::string::npos) return fail(PPM_EINVAL, "tile_config: bad token '%s'", tok.c_str());
    const std::string k = tok.substr(0, eq);
    char *end = nullptr;
    const long v = strtol(tok.c_str() + eq + 1, &end, 10);
    if (!end || *end) return fail(PPM_EINVAL, "tile_config: bad value in '%s'", tok.c_str());
    if (k == "block") {
      if (v < 64 || v > ppm::kMaxBlock || v % 64) return fail(PPM_EINVAL, "tile_config: block must be 64..256, a multiple of 64");
      pl->block = int32_t(v);
      pl->lanes_set = true;
    } else if (k == "lanes") {
      if (v < 0 || v > 7) return fail(PPM_EINVAL, "tile_config: lanes is an axis bitmask 0..7");
      pl->lanes_mask = int32_t(v);
      pl->lanes_set = true;
    } else if (k == "lanes_block") {
      if (v < 64 || v > ppm::kMaxBlock || v % 64) return fail(PPM_EINVAL, "tile_config: lanes_block must be 64..256, a multiple of 64");
      pl->lanes_block = int32_t(v);
    } else if (k == "group") {
      if (v != 0 && v != 1) return fail(PPM_EINVAL, "tile_config: group must be 0 or 1");
      pl->group = int32_t(v);
      pl->group_set = true;
    } else if (k == "tail") {
      if (v != 0 && v != 1) return fail(PPM_EINVAL, "tile_config: tail must be 0 or 1");
      pl->tail = int32_t(v);
      pl->lanes_set = true;
    } else if (k == "split") {
      if (v != 0 && v != 1) return fail(PPM_EINVAL, "tile_config: split must be 0 or 1");
      pl->split = int32_t(v);
    } else if (k == "tail_round") {
      if (v < 64 || v > (1 << 26) || v % 64) return fail(PPM_EINVAL, "tile_config: tail_round must be a multiple of 64 in 64..2^26");
      pl->tail_round = int32_t(v);
      pl->lanes_set = true;
    } else if (k == "persistent") {
      if (v != 0 && v != 1) return fail(PPM_EINVAL, "tile_config: persistent must be 0 or 1");
      pl->persistent = int32_t(v);
    } else if (k == "batch_block") {
      if (v < 64 || v > ppm::kMaxBlock || v % 64) return fail(PPM_EINVAL, "tile_config: batch_block must be 64..256, a multiple of 64");
      pl->batch_block = int32_t(v);
    } else if (k == "batch_blocks") {
      if (v < 1 || v > (1 << 20)) return fail(PPM_EINVAL, "tile_config: batch_blocks out of range");
      pl->batch_blocks = int32_t(v);
    } else if (k == "cfl_cells") {
      if (v < 256 || v > (1 << 24)) return fail(PPM_EINVAL, "tile_config: cfl_cells out of range");
      pl->cfl_cells = int32_t(v);
    } else {
      return fail(PPM_EINVAL, "tile_config: unknown key '%s'", k.c_str());
    }
  }
  return PPM_OK;
}

void free_plan(ppm_plan *p) {
  if (!p) return;
  if (p->d_patches) (void)hipFree(p->d_patches);
  if (p->d_chunks) (void)hipFree(p->d_chunks);
  if (p->d_counters) (void)hipFree(p->d_counters);
  if (p->d_smax) (void)hipFree(p->d_smax);
  if (p->d_order) (void)hipFree(p->d_order);
  if (p->d_defer) (void)hipFree(p->d_defer);
  if (p->d_queue) (void)hipFree(p->d_queue);
  if (p->d_groups) (void)hipFree(p->d_groups);
  if (p->d_interp) (void)hipFree(p->d_interp);
  if (p->d_boxes) (void)hipFree(p->d_boxes);
  if (p->d_iprefix) (void)hipFree(p->d_iprefix);
  if (p->d_bprefix) (void)hipFree(p->d_bprefix);
  delete p;
}

// One sweep over every patch; smax (nullable): also take the max signal
// speed per level of the cells written.
template <class Prec>
hipError_t do_sweep(ppm_plan *pl, const double *dt, int axis, int mask, unsigned long long *smax,
                    hipStream_t s) {
  const int tm = tmask_of(axis, mask);
  if ((pl->lanes_mask >> axis) & 1) {
    const int slot = 12 + axis * 4 + tm;
    if (pl->nblocks[slot] == 0) return hipSuccess;
    return ppm::launch_sweep_lanes<Prec>(pl->d_patches, pl->d_chunks + slot * (pl->npatch + 1),
                                         pl->npatch, pl->nblocks[slot], pl->lanes_block, axis,
                                         mask, dt, pl->P, pl->d_counters, smax, s);
  }
  const int slot = axis * 4 + tm;
  if (pl->nblocks[slot] == 0) return hipSuccess;
  const int32_t *groups = pl->group ? pl->d_groups + pl->gofs[slot] : nullptr;
  const int c = smax ? 1 : 0;
  const int32_t *chunks = pl->d_chunks + slot * (pl->npatch + 1);
  double *defer = pl->split_on[c][slot] ? pl->d_defer : nullptr;
  if (pl->tail_blocks[c][slot] > 0) {  // whole rounds marched, the rest one pencil per wave
    hipError_t e = ppm::launch_sweep<Prec>(pl->d_patches, chunks, pl->npatch,
                                           pl->tail_main[c][slot], pl->block, axis, mask, dt,
                                           pl->P, pl->d_counters, smax, nullptr, 0, s, defer);
    if (e != hipSuccess) return e;
    return ppm::launch_sweep_tail<Prec>(pl->d_patches, chunks, pl->tail_blocks[c][slot],
                                        pl->lanes_block, axis, mask, pl->tail_pencil0[c][slot],
                                        dt, pl->P, pl->d_counters, smax, s);
  }
  if (defer)
    return ppm::launch_sweep<Prec>(pl->d_patches, chunks, pl->npatch, pl->split_blocks[c][slot],
                                   pl->block, axis, mask, dt, pl->P, pl->d_counters, smax,
                                   nullptr, 0, s, defer);
  return ppm::launch_sweep<Prec>(pl->d_patches, chunks, pl->npatch, pl->nblocks[slot], pl->block,
                                 axis, mask, dt, pl->P, pl->d_counters, smax, groups,
                                 pl->ngroups[slot], s);
}

hipError_t sweep_any(ppm_plan *pl, const double *dt, int axis, int mask, unsigned long long *smax,
                     hipStream_t s) {
  return pl->prec == PPM_FP64 ? do_sweep<ppm::PrecF64>(pl, dt, axis, mask, smax, s)
                              : do_sweep<ppm::PrecMixed>(pl, dt, axis, mask, smax, s);
}

}  // namespace

extern "C" {

ppm_status ppm_fp64_ops(const double *a_dev, const double *b_dev, double *quot_dev,
                        double *root_dev, int64_t n, void *hip_stream) {
  if (n < 0 || n > (int64_t(1) << 36)) return fail(PPM_EINVAL, "n must be in [0, 2^36]");
  if (n > 0 && (!a_dev || !b_dev || !quot_dev || !root_dev))
    return fail(PPM_EINVAL, "NULL array");
  const hipError_t e = ppm::launch_fp64_ops(a_dev, b_dev, quot_dev, root_dev, n,
                                            static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? PPM_OK : hip_fail(e, "ppm_fp64_ops");
}

int64_t ppm_flux_reg_size(int32_t nx, int32_t ny, int32_t nz) {
  return 12 * (int64_t(ny) * nz + int64_t(nx) * nz + int64_t(nx) * ny);
}

ppm_status ppm_plan_create(ppm_plan **out, const ppm_patch *patches, int32_t npatch,
                           int32_t nlevels, ppm_precision prec, const ppm_params *params,
                           const char *tile_config, void *hip_stream) {
  if (!out) return fail(PPM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!patches) return fail(PPM_EINVAL, "patches is NULL");
  if (npatch < 1) return fail(PPM_EINVAL, "npatch must be >= 1");
  if (nlevels < 1 || nlevels > 64) return fail(PPM_EINVAL, "nlevels must be in 1..64");
  if (prec != PPM_FP64 && prec != PPM_MIXED) return fail(PPM_EINVAL, "unknown precision %d", int(prec));
  ppm_status st = check_params(params);
  if (st != PPM_OK) return st;
  if ((st = ppm_detail::check_mixed_floors(prec, params)) != PPM_OK) return st;
  for (int i = 0; i < npatch; ++i)
    if ((st = check_patch(patches[i], i, nlevels)) != PPM_OK) return st;

  ppm_plan *pl = new (std::nothrow) ppm_plan();
  if (!pl) return fail(PPM_ENOMEM, "host allocation failed");
  pl->npatch = npatch;
  pl->nlevels = nlevels;
  pl->prec = prec;
  pl->P = ppm_detail::device_params(prec, params);
  int64_t max_cells = 0;
  for (int i = 0; i < npatch; ++i)
    max_cells = std::max(max_cells, int64_t(patches[i].nx) * patches[i].ny * patches[i].nz);
  if (npatch > 1) {  // uneven patches: finer chunks, one persistent launch if they are small
    pl->block = 64;
    pl->lanes_block = 64;
    pl->persistent = max_cells <= kPersistentMaxCells ? 1 : 0;
    pl->group = 1;
  }
  if ((st = parse_tiles(pl, tile_config)) != PPM_OK) {
    delete pl;
    return st;
  }
  if (pl->tail_round % pl->block) {
    delete pl;
    return fail(PPM_EINVAL, "tile_config: tail_round must be a multiple of block");
  }
  if (pl->persistent && max_cells > kPersistentMaxCells) {
    delete pl;
    return fail(PPM_EINVAL, "persistent=1 needs every patch to hold at most %lld active cells",
                (long long)kPersistentMaxCells);
  }
  (void)hipGetDevice(&pl->device);
  // One small patch: a marching sweep would give each of its few pencils a
  // thread and leave most of the device idle (a 128^3 grid's y sweep has
  // 134^2 pencils for 2 x 256 resident threads on each of 256 CUs), so every
  // sweep streams its pencils through the lanes instead (measured: 128^3 FP64
  // 1.80 -> 1.25 ms per step; from 192^3 on the marching sweeps are faster).
  if (npatch == 1 && !pl->lanes_set) {
    int cus0 = 0;
    if (hipDeviceGetAttribute(&cus0, hipDeviceAttributeMultiprocessorCount, pl->device) !=
        hipSuccess)
      cus0 = 0;
    const ppm_patch &q = patches[0];
    const int64_t pencils = (int64_t(q.nx) + 2 * q.ghost) * (int64_t(q.nz) + 2 * q.ghost);
    if (cus0 > 0 && pencils * 8 < int64_t(cus0) * 2 * 256 * 2) pl->lanes_mask = 7;
  }
  pl->host.resize(npatch);
  pl->bc.resize(npatch);
  for (int i = 0; i < npatch; ++i) pl->bc[i] = patches[i].bc;
  for (int i = 0; i < npatch; ++i) {
    const ppm_patch &q = patches[i];
    PatchDev &d = pl->host[i];
    d.n[0] = q.nx; d.n[1] = q.ny; d.n[2] = q.nz;
    d.ghost = q.ghost; d.level = q.level; d.pad = 0;
    d.dx[0] = q.dx; d.dx[1] = q.dy; d.dx[2] = q.dz;
    d.rho = q.rho; d.vel[0] = q.vx; d.vel[1] = q.vy; d.vel[2] = q.vz;
    d.etot = q.etot; d.eint = q.eint; d.flux_reg = q.flux_reg;
    d.acc[0] = q.gx; d.acc[1] = q.gy; d.acc[2] = q.gz;
    if (q.gx) pl->P.flags |= ppm::kAnyGravity;
  }
  // prefix arrays of work chunks
  const int stride = npatch + 1;
  std::vector<int32_t> chunks(size_t(25) * stride, 0);
  for (int kind = 0; kind < 2; ++kind)  // 0: marching (a thread per pencil), 1: lanes
    for (int axis = 0; axis < 3; ++axis)
      for (int tm = 0; tm < 4; ++tm) {
        const int slot = kind * 12 + axis * 4 + tm;
        int64_t acc = 0;
        int32_t *c = &chunks[size_t(slot) * stride];
        const int t1 = t1_of(axis), t2 = t2_of(axis);
        for (int i = 0; i < npatch; ++i) {
          const PatchDev &d = pl->host[i];
          const int64_t w1 = (tm & 1) ? d.n[t1] : d.n[t1] + 2 * d.ghost;
          const int64_t w2 = (tm & 2) ? d.n[t2] : d.n[t2] + 2 * d.ghost;
          // work items: pencils (marching), or waves streaming runs of pencils
          // (lane-parallel)
          int64_t items = w1 * w2, per_block = pl->block;
          if (kind == 1) {  // a wave streams rows_per_wave(n) pencils
            const int64_t rpw = ppm::rows_per_wave(int(d.n[axis] + 2 * d.ghost));
            items = (items + rpw - 1) / rpw;
            per_block = pl->lanes_block / 64;
          }
          c[i] = int32_t(acc);
          acc += (items + per_block - 1) / per_block;
          if (acc > std::numeric_limits<int32_t>::max() / 2) {
            delete pl;
            return fail(PPM_EINVAL, "too many pencils for one launch");
          }
        }
        c[npatch] = int32_t(acc);
        pl->nblocks[slot] = int32_t(acc);
      }
  // grouped marching maps: per (axis, extent) slot, the patches sorted by
  // pencil length, longest first (the last blocks to start then hold the
  // shortest pencils), runs of equal length, the first block of each run, the
  // first sorted patch of each run, the pencil prefix over the sorted patches
  // and the sorted patch indices
  // A run's patches must be views into six shared arrays at one element
  // offset per patch (the run's first patch lends its field pointers to the
  // whole wave).
  auto aligned = [&](int i, int r) {
    const ppm_patch &q = patches[i], &b = patches[r];
    const int64_t sS = prec == PPM_FP64 ? 8 : 4;
    auto d = [](const void *x, const void *y) {
      return int64_t(reinterpret_cast<uintptr_t>(x)) - int64_t(reinterpret_cast<uintptr_t>(y));
    };
    const int64_t dr = d(q.rho, b.rho);
    const bool qg = q.gx != nullptr, bg = b.gx != nullptr;
    return dr % sS == 0 && d(q.vx, b.vx) == dr && d(q.vy, b.vy) == dr && d(q.vz, b.vz) == dr &&
           d(q.etot, b.etot) == dr / sS * 8 && d(q.eint, b.eint) == dr / sS * 8 && qg == bg &&
           (!qg || (d(q.gx, b.gx) == dr && d(q.gy, b.gy) == dr && d(q.gz, b.gz) == dr));
  };
  std::vector<int32_t> gmap;
  bool runs_aligned = true;
  if (pl->group) {
    for (int axis = 0; axis < 3; ++axis)
      for (int tm = 0; tm < 4; ++tm) {
        const int slot = axis * 4 + tm;
        const int t1 = t1_of(axis), t2 = t2_of(axis);
        std::vector<int32_t> sorted(npatch);
        for (int i = 0; i < npatch; ++i) sorted[i] = i;
        auto len = [&](int i) { return pl->host[i].n[axis] + 2 * pl->host[i].ghost; };
        std::stable_sort(sorted.begin(), sorted.end(),
                         [&](int a, int b) { return len(a) > len(b); });
        std::vector<int32_t> pp(size_t(npatch) + 1, 0), gfirst, gbs;
        int64_t acc = 0, blocks = 0;
        for (int j = 0; j < npatch; ++j) {
          const PatchDev &d = pl->host[sorted[j]];
          const int64_t w1 = (tm & 1) ? d.n[t1] : d.n[t1] + 2 * d.ghost;
          const int64_t w2 = (tm & 2) ? d.n[t2] : d.n[t2] + 2 * d.ghost;
          if (j == 0 || len(sorted[j]) != len(sorted[j - 1])) {
            if (j > 0) blocks += (acc - pp[gfirst.back()] + pl->block - 1) / pl->block;
            gfirst.push_back(j);
            gbs.push_back(int32_t(blocks));
          }
          runs_aligned = runs_aligned && aligned(sorted[j], sorted[gfirst.back()]);
          pp[j] = int32_t(acc);
          acc += w1 * w2;
          if (acc > std::numeric_limits<int32_t>::max() / 2) {
            delete pl;
            return fail(PPM_EINVAL, "too many pencils for one launch");
          }
        }
        pp[npatch] = int32_t(acc);
        blocks += (acc - pp[gfirst.back()] + pl->block - 1) / pl->block;
        gfirst.push_back(npatch);
        gbs.push_back(int32_t(blocks));
        pl->ngroups[slot] = int32_t(gfirst.size()) - 1;
        pl->nblocks[slot] = int32_t(blocks);
        pl->gofs[slot] = int64_t(gmap.size());
        gmap.insert(gmap.end(), gbs.begin(), gbs.end());
        gmap.insert(gmap.end(), gfirst.begin(), gfirst.end());
        gmap.insert(gmap.end(), pp.begin(), pp.end());
        gmap.insert(gmap.end(), sorted.begin(), sorted.end());
      }
    if (!runs_aligned) {
      if (pl->group_set) {
        delete pl;
        return fail(PPM_EINVAL, "tile_config: group=1 needs the patches of equal pencil length to "
                                "be views at one element offset into six shared arrays");
      }
      pl->group = 0;  // per-patch launch maps (the marching block counts above)
      gmap.clear();
      for (int slot = 0; slot < 12; ++slot)
        pl->nblocks[slot] = chunks[size_t(slot + 1) * stride - 1];
    }
  }
  // One patch, few pencils: a marching sweep with fewer pencils than two
  // blocks per compute unit leaves the device at one wave per SIMD or less,
  // so two threads march each pencil (split; pencils of at least 16 active
  // cells).  And marched threads just over a whole number of rounds of one
  // block per compute unit: march the whole rounds and give the few pencils
  // left (at most an eighth of a round) to the lane-parallel kernel, one
  // pencil per wave, instead of a last round in which a few compute units
  // march a block more than the others (a 256^3 y sweep: 262 blocks of 256
  // on 256 compute units took 2.2 ms, the 256 blocks of its z sweep 1.55).
  // A given tail_round replaces the round and the eighth rule (any rest).
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl->device) != hipSuccess)
    cus = 0;
  int64_t defer_pencils = 0;
  if (npatch == 1 && !pl->group && (cus > 0 || pl->tail_round > 0)) {
    for (int c = 0; c < 2; ++c) {
      for (int slot = 0; slot < 12; ++slot) {
        const int axis = slot / 4, tm = slot % 4;
        const PatchDev &d = pl->host[0];
        const int64_t w1 = (tm & 1) ? d.n[t1_of(axis)] : d.n[t1_of(axis)] + 2 * d.ghost;
        const int64_t w2 = (tm & 2) ? d.n[t2_of(axis)] : d.n[t2_of(axis)] + 2 * d.ghost;
        const int64_t np = w1 * w2;
        const bool split = pl->split && cus > 0 && d.n[axis] >= 16 &&
                           np < 2 * int64_t(cus) * pl->block;
        const int64_t tpp = split ? 2 : 1, threads = tpp * np;
        // threads per round: tail_round pencils, else one block per compute unit
        const int64_t cap = pl->tail_round ? pl->tail_round * tpp : int64_t(cus) * pl->block;
        if (split) {
          pl->split_on[c][slot] = 1;
          pl->split_blocks[c][slot] = int32_t((threads + pl->block - 1) / pl->block);
          defer_pencils = std::max(defer_pencils, np);
        }
        if (!pl->tail || cap <= 0) continue;
        const int64_t rest = threads % cap;
        if (threads < cap || rest == 0 || (pl->tail_round == 0 && rest * 8 > cap)) continue;
        const int64_t waves = pl->lanes_block / 64;
        pl->tail_pencil0[c][slot] = int32_t((threads - rest) / tpp);
        pl->tail_main[c][slot] = int32_t((threads - rest) / pl->block);
        pl->tail_blocks[c][slot] = int32_t((rest / tpp + waves - 1) / waves);
      }
    }
  }
  {
    int64_t acc = 0;
    int32_t *c = &chunks[size_t(24) * stride];
    for (int i = 0; i < npatch; ++i) {
      const PatchDev &d = pl->host[i];
      const int64_t cells = int64_t(d.n[0]) * d.n[1] * d.n[2];
      c[i] = int32_t(acc);
      acc += (cells + pl->cfl_cells - 1) / pl->cfl_cells;
      if (acc > std::numeric_limits<int32_t>::max() / 2) {
        delete pl;
        return fail(PPM_EINVAL, "too many cells for one CFL launch");
      }
    }
    c[npatch] = int32_t(acc);
    pl->cfl_blocks = int32_t(acc);
  }
  // persistent queue order: descending cost (cell-sweeps of a step)
  std::vector<int32_t> order(npatch);
  {
    std::vector<std::pair<double, int32_t>> cost(npatch);
    for (int i = 0; i < npatch; ++i) {
      const PatchDev &d = pl->host[i];
      const double a = d.n[0], b = d.n[1], c = d.n[2], g2 = 2.0 * d.ghost;
      cost[i] = {-(a * (b + g2) * (c + g2) + a * b * (c + g2) + a * b * c), i};
    }
    std::stable_sort(cost.begin(), cost.end());
    for (int i = 0; i < npatch; ++i) order[i] = cost[i].second;
  }
  if (pl->batch_blocks == 0)
    pl->batch_blocks = std::min<int64_t>(int64_t(cus > 0 ? cus : 256) * (512 / pl->batch_block),
                                         npatch);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e;
  if ((e = hipMalloc(&pl->d_order, sizeof(int32_t) * npatch)) != hipSuccess ||
      (e = hipMalloc(&pl->d_queue, 2 * sizeof(unsigned int))) != hipSuccess ||
      (e = hipMalloc(&pl->d_patches, sizeof(PatchDev) * npatch)) != hipSuccess ||
      (e = hipMalloc(&pl->d_chunks, sizeof(int32_t) * chunks.size())) != hipSuccess ||
      (e = hipMalloc(&pl->d_counters, 2 * sizeof(unsigned long long))) != hipSuccess ||
      (e = hipMalloc(&pl->d_smax, nlevels * sizeof(unsigned long long))) != hipSuccess ||
      (!gmap.empty() &&
       (e = hipMalloc(&pl->d_groups, sizeof(int32_t) * gmap.size())) != hipSuccess) ||
      (defer_pencils > 0 &&
       (e = hipMalloc(&pl->d_defer, sizeof(double) * size_t(defer_pencils) * 30)) !=
           hipSuccess)) {
    free_plan(pl);
    return fail(PPM_ENOMEM, "hipMalloc: %s", hipGetErrorString(e));
  }
  std::vector<unsigned long long> zeros(size_t(nlevels) + 2, 0ull);
  if ((e = hipMemcpyAsync(pl->d_order, order.data(), sizeof(int32_t) * npatch,
                          hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(pl->d_queue, zeros.data(), 2 * sizeof(unsigned int),
                          hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(pl->d_patches, pl->host.data(), sizeof(PatchDev) * npatch,
                          hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(pl->d_chunks, chunks.data(), sizeof(int32_t) * chunks.size(),
                          hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(pl->d_counters, zeros.data(), 2 * sizeof(unsigned long long),
                          hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(pl->d_smax, zeros.data(), nlevels * sizeof(unsigned long long),
                          hipMemcpyHostToDevice, s)) != hipSuccess ||
      (!gmap.empty() &&
       (e = hipMemcpyAsync(pl->d_groups, gmap.data(), sizeof(int32_t) * gmap.size(),
                           hipMemcpyHostToDevice, s)) != hipSuccess) ||
      (e = hipStreamSynchronize(s)) != hipSuccess) {
    free_plan(pl);
    return hip_fail(e, "plan upload");
  }
  *out = pl;
  return PPM_OK;
}

ppm_status ppm_plan_destroy(ppm_plan *plan) {
  free_plan(plan);
  return PPM_OK;
}

ppm_status ppm_fill_periodic(ppm_plan *plan, void *hip_stream) {
  if (!plan) return fail(PPM_EINVAL, "plan is NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  for (int i = 0; i < plan->npatch; ++i) {
    if (plan->bc[i] != PPM_BC_PERIODIC) continue;
    hipError_t e = plan->prec == PPM_FP64 ? ppm::launch_fill<ppm::PrecF64>(plan->host[i], s)
                                          : ppm::launch_fill<ppm::PrecMixed>(plan->host[i], s);
    if (e != hipSuccess) return hip_fail(e, "fill_periodic launch");
  }
  return PPM_OK;
}

ppm_status ppm_fill_boundary(ppm_plan *plan, int32_t patch, const int32_t *kinds,
                             const double *inflow, void *hip_stream) {
  if (!plan) return fail(PPM_EINVAL, "plan is NULL");
  if (patch < 0 || patch >= plan->npatch)
    return fail(PPM_EINVAL, "patch %d outside [0, %d)", patch, plan->npatch);
  if (!kinds) return fail(PPM_EINVAL, "kinds is NULL");
  const PatchDev &pd = plan->host[patch];
  ppm::FaceRules fr{};
  for (int f = 0; f < 6; ++f) {
    const int32_t k = kinds[f];
    if (k < PPM_FACE_PERIODIC || k > PPM_FACE_INFLOW)
      return fail(PPM_EINVAL, "face %d: unknown boundary kind %d", f, k);
    if (k == PPM_FACE_INFLOW && !inflow)
      return fail(PPM_EINVAL, "face %d is PPM_FACE_INFLOW but inflow is NULL", f);
    if (k == PPM_FACE_REFLECTING && pd.n[f / 2] < pd.ghost)
      return fail(PPM_EINVAL, "face %d: reflecting needs at least %d active cells", f, pd.ghost);
    fr.kind[f] = k;
    if (k == PPM_FACE_INFLOW)
      for (int q = 0; q < 6; ++q) fr.inflow[f][q] = inflow[f * 6 + q];
  }
  for (int a = 0; a < 3; ++a)
    if ((kinds[2 * a] == PPM_FACE_PERIODIC) != (kinds[2 * a + 1] == PPM_FACE_PERIODIC))
      return fail(PPM_EINVAL, "axis %d: periodic faces come in pairs", a);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = plan->prec == PPM_FP64 ? ppm::launch_fill_boundary<ppm::PrecF64>(pd, fr, s)
                                        : ppm::launch_fill_boundary<ppm::PrecMixed>(pd, fr, s);
  if (e != hipSuccess) return hip_fail(e, "fill_boundary launch");
  return PPM_OK;
}

namespace {
int64_t floor_div64(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
// Parent cells (in the parent's level) whose r^3 fine cells meet the box
// [lo, hi) of local (ghosted) cells of a patch that starts at `start` of its
// level: one thread each in the parent-interpolation launch.
int64_t parent_box_count(const PatchDev &d, const int32_t start[3], int32_t r,
                         const int32_t lo[3], const int32_t hi[3]) {
  int64_t v = 1;
  for (int a = 0; a < 3; ++a) {
    const int64_t c0 = floor_div64(int64_t(start[a]) + lo[a] - d.ghost, r);
    const int64_t c1 = floor_div64(int64_t(start[a]) + hi[a] - 1 - d.ghost, r);
    v *= c1 - c0 + 1;
  }
  return v;
}
// The ghost cells of a patch as six disjoint slabs of local (ghosted)
// indices: below and above the active cells along z (whole x-y planes), then
// along y (active z), then along x (active y and z).
void ghost_slabs(const PatchDev &d, std::vector<ppm_detail::IBox> &v) {
  const int64_t g = d.ghost;
  v.clear();
  for (int a = 2; a >= 0; --a)
    for (int side = 0; side < 2; ++side) {
      ppm_detail::IBox b{};
      for (int k = 0; k < 3; ++k) {
        const int64_t n = d.n[k];
        if (k == a) {
          b.lo[k] = side ? g + n : 0;
          b.hi[k] = side ? n + 2 * g : g;
        } else if (k > a) {
          b.lo[k] = g; b.hi[k] = g + n;
        } else {
          b.lo[k] = 0; b.hi[k] = n + 2 * g;
        }
      }
      if (b.volume() > 0) v.push_back(b);
    }
}
}  // namespace

ppm_status ppm_set_hierarchy(ppm_plan *plan, const ppm_patch_place *place, void *hip_stream) {
  if (!plan) return fail(PPM_EINVAL, "plan is NULL");
  if (!place) return fail(PPM_EINVAL, "place is NULL");
  const int np = plan->npatch, nl = plan->nlevels;
  const auto &H = plan->host;
  for (int i = 0; i < np; ++i) {
    const ppm_patch_place &q = place[i];
    if (q.parent < 0) continue;
    if (q.parent >= np) return fail(PPM_EINVAL, "patch %d: parent %d out of range", i, q.parent);
    if (H[q.parent].level != H[i].level - 1)
      return fail(PPM_EINVAL, "patch %d: parent %d is not one level coarser", i, q.parent);
    if (q.refine < 2) return fail(PPM_EINVAL, "patch %d: refine must be >= 2", i);
    const PatchDev &f = H[i], &c = H[q.parent];
    const ppm_patch_place &pp = place[q.parent];
    for (int a = 0; a < 3; ++a) {
      const int64_t lo = floor_div64(int64_t(q.start[a]) - f.ghost, q.refine) - pp.start[a] + c.ghost;
      const int64_t hi = floor_div64(int64_t(q.start[a]) + f.n[a] + f.ghost - 1, q.refine) -
                         pp.start[a] + c.ghost;
      if (lo < 1 || hi > int64_t(c.n[a]) + 2 * c.ghost - 2)
        return fail(PPM_EINVAL, "patch %d: its ghost cells need parent cells outside parent %d "
                                "(axis %d)", i, q.parent, a);
    }
  }
  // sibling boxes, and the ghost cells that no sibling covers, which the
  // parent interpolation fills (the others would be overwritten by the
  // sibling copies that follow it), grouped by level
  std::vector<ppm::InterpItem> items;
  std::vector<ppm::SiblingBox> boxes;
  std::vector<int64_t> ipre, bpre;
  std::vector<int32_t> ibeg(nl + 1, 0), bbeg(nl + 1, 0);
  std::vector<int64_t> itot(nl, 0), btot(nl, 0);
  std::vector<std::vector<int>> bylevel(nl);
  for (int i = 0; i < np; ++i) bylevel[H[i].level].push_back(i);
  std::vector<std::vector<ppm_detail::IBox>> uncovered(np);
  for (int L = 0; L < nl; ++L) {
    bbeg[L] = int32_t(boxes.size());
    int64_t bacc = 0;
    for (int d : bylevel[L]) {
      if (place[d].parent < 0) continue;
      ghost_slabs(H[d], uncovered[d]);
      for (int src : bylevel[L]) {
        if (src == d) continue;
        ppm::SiblingBox b{};
        b.dst = d; b.src = src;
        bool empty = false;
        for (int a = 0; a < 3; ++a) {
          const int64_t g = H[d].ghost;
          const int64_t lo = std::max<int64_t>(int64_t(place[d].start[a]) - g, place[src].start[a]);
          const int64_t hi = std::min<int64_t>(int64_t(place[d].start[a]) + H[d].n[a] + g,
                                               int64_t(place[src].start[a]) + H[src].n[a]);
          if (lo >= hi) { empty = true; break; }
          b.lo[a] = int32_t(lo - place[d].start[a] + g);
          b.hi[a] = int32_t(hi - place[d].start[a] + g);
          b.shift[a] = int32_t(int64_t(place[d].start[a]) - g - place[src].start[a] + H[src].ghost);
        }
        if (empty) continue;
        boxes.push_back(b);
        bpre.push_back(bacc);
        bacc += int64_t(b.hi[0] - b.lo[0]) * (b.hi[1] - b.lo[1]) * (b.hi[2] - b.lo[2]);
        ppm_detail::boxes_minus(uncovered[d], ppm_detail::IBox{{b.lo[0], b.lo[1], b.lo[2]},
                                                               {b.hi[0], b.hi[1], b.hi[2]}});
      }
    }
    bpre.push_back(bacc);
    btot[L] = bacc;
  }
  for (int L = 0; L < nl; ++L) {
    ibeg[L] = int32_t(items.size());
    int64_t acc = 0;
    for (int i : bylevel[L]) {
      if (place[i].parent < 0) continue;
      for (const ppm_detail::IBox &u : uncovered[i]) {
        ppm::InterpItem it{};
        it.patch = i; it.parent = place[i].parent; it.r = place[i].refine;
        for (int a = 0; a < 3; ++a) {
          it.start[a] = place[i].start[a];
          it.pstart[a] = place[place[i].parent].start[a];
          it.lo[a] = int32_t(u.lo[a]);
          it.hi[a] = int32_t(u.hi[a]);
        }
        items.push_back(it);
        ipre.push_back(acc);
        acc += parent_box_count(H[i], it.start, it.r, it.lo, it.hi);
      }
    }
    ipre.push_back(acc);
    itot[L] = acc;
  }
  ibeg[nl] = int32_t(items.size());
  bbeg[nl] = int32_t(boxes.size());
  // replace the device lists
  if (plan->d_interp) (void)hipFree(plan->d_interp);
  if (plan->d_boxes) (void)hipFree(plan->d_boxes);
  if (plan->d_iprefix) (void)hipFree(plan->d_iprefix);
  if (plan->d_bprefix) (void)hipFree(plan->d_bprefix);
  plan->d_interp = nullptr; plan->d_boxes = nullptr;
  plan->d_iprefix = plan->d_bprefix = nullptr;
  plan->hier = false;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e;
  auto up = [&](void **dst, const void *src, size_t bytes) -> hipError_t {
    hipError_t r = hipMalloc(dst, bytes ? bytes : 8);
    if (r != hipSuccess) return r;
    return bytes ? hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
  };
  if ((e = up((void **)&plan->d_interp, items.data(), items.size() * sizeof(ppm::InterpItem))) !=
          hipSuccess ||
      (e = up((void **)&plan->d_boxes, boxes.data(), boxes.size() * sizeof(ppm::SiblingBox))) !=
          hipSuccess ||
      (e = up((void **)&plan->d_iprefix, ipre.data(), ipre.size() * sizeof(int64_t))) != hipSuccess ||
      (e = up((void **)&plan->d_bprefix, bpre.data(), bpre.size() * sizeof(int64_t))) != hipSuccess)
    return hip_fail(e, "hierarchy upload");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hierarchy upload");
  plan->ibeg = ibeg; plan->bbeg = bbeg; plan->itotal = itot; plan->btotal = btot;
  plan->h_interp = std::move(items);
  plan->hier = true;
  return PPM_OK;
}

ppm_status ppm_fill_ghosts(ppm_plan *plan, int32_t level, void *hip_stream) {
  return ppm_detail::fill_ghosts(plan, level, nullptr, static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"

void ppm_detail::boxes_minus(std::vector<IBox> &list, const IBox &b) {
  std::vector<IBox> out;
  out.reserve(list.size() + 6);
  for (IBox a : list) {
    bool meets = true;
    for (int k = 0; k < 3; ++k) meets = meets && a.lo[k] < b.hi[k] && b.lo[k] < a.hi[k];
    if (!meets) {
      out.push_back(a);
      continue;
    }
    // peel off the parts below and above b along each axis in turn; what
    // remains of a lies inside b
    for (int k = 0; k < 3; ++k) {
      if (a.lo[k] < b.lo[k]) {
        IBox piece = a;
        piece.hi[k] = b.lo[k];
        out.push_back(piece);
        a.lo[k] = b.lo[k];
      }
      if (a.hi[k] > b.hi[k]) {
        IBox piece = a;
        piece.lo[k] = b.hi[k];
        out.push_back(piece);
        a.hi[k] = b.hi[k];
      }
    }
  }
  list.swap(out);
}

ppm_status ppm_detail::fill_ghosts(ppm_plan *plan, int32_t level, const PatchDev *parent_tab,
                                   hipStream_t s) {
  if (!plan) return fail(PPM_EINVAL, "plan is NULL");
  if (!plan->hier) return fail(PPM_EINVAL, "no hierarchy recorded (ppm_set_hierarchy)");
  if (level < 0 || level >= plan->nlevels)
    return fail(PPM_EINVAL, "level %d outside [0, %d)", level, plan->nlevels);
  const int32_t i0 = plan->ibeg[level], ni = plan->ibeg[level + 1] - i0;
  const int32_t b0 = plan->bbeg[level], nb = plan->bbeg[level + 1] - b0;
  // prefix arrays hold one extra entry per level before it
  const int64_t *ip = plan->d_iprefix + i0 + level;
  const int64_t *bp = plan->d_bprefix + b0 + level;
  hipError_t e;
  if (ni > 0) {
    e = plan->prec == PPM_FP64
        ? ppm::launch_fill_from_parent<ppm::PrecF64>(plan->d_patches, plan->d_interp + i0, ip, ni,
                                                     plan->itotal[level], parent_tab, s)
        : ppm::launch_fill_from_parent<ppm::PrecMixed>(plan->d_patches, plan->d_interp + i0, ip,
                                                       ni, plan->itotal[level], parent_tab, s);
    if (e != hipSuccess) return hip_fail(e, "fill_from_parent launch");
  }
  if (nb > 0) {
    e = plan->prec == PPM_FP64
        ? ppm::launch_copy_from_siblings<ppm::PrecF64>(plan->d_patches, plan->d_boxes + b0, bp, nb,
                                                       plan->btotal[level], s)
        : ppm::launch_copy_from_siblings<ppm::PrecMixed>(plan->d_patches, plan->d_boxes + b0, bp,
                                                         nb, plan->btotal[level], s);
    if (e != hipSuccess) return hip_fail(e, "copy_from_siblings launch");
  }
  return PPM_OK;
}

extern "C" {

ppm_status ppm_set_expansion(ppm_plan *plan, const double *a_dev) {
  if (!plan) return fail(PPM_EINVAL, "plan is NULL");
  plan->P.expand = a_dev;
  return PPM_OK;
}

ppm_status ppm_expansion(ppm_plan *plan, const double *dt_dev, void *hip_stream) {
  if (!plan) return fail(PPM_EINVAL, "plan is NULL");
  if (!dt_dev) return fail(PPM_EINVAL, "dt_dev is NULL");
  if (!plan->P.expand) return fail(PPM_EINVAL, "no expansion factors set (ppm_set_expansion)");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int32_t *cs = plan->d_chunks + size_t(24) * (plan->npatch + 1);
  hipError_t e = plan->prec == PPM_FP64
      ? ppm::launch_expansion<ppm::PrecF64>(plan->d_patches, cs, plan->npatch, plan->cfl_blocks,
                                            plan->cfl_cells, plan->P.gamma, plan->P.expand,
                                            dt_dev, s)
      : ppm::launch_expansion<ppm::PrecMixed>(plan->d_patches, cs, plan->npatch,
                                              plan->cfl_blocks, plan->cfl_cells, plan->P.gamma,
                                              plan->P.expand, dt_dev, s);
  if (e != hipSuccess) return hip_fail(e, "expansion launch");
  return PPM_OK;
}

ppm_status ppm_cfl_dt(ppm_plan *plan, double *dt_dev, void *hip_stream) {
  if (!plan) return fail(PPM_EINVAL, "plan is NULL");
  if (!dt_dev) return fail(PPM_EINVAL, "dt_dev is NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int32_t *cs = plan->d_chunks + size_t(24) * (plan->npatch + 1);
  hipError_t e = plan->prec == PPM_FP64
      ? ppm::launch_cfl<ppm::PrecF64>(plan->d_patches, cs, plan->npatch, plan->cfl_blocks,
                                      plan->cfl_cells, plan->nlevels, plan->P, plan->d_smax,
                                      dt_dev, s)
      : ppm::launch_cfl<ppm::PrecMixed>(plan->d_patches, cs, plan->npatch, plan->cfl_blocks,
                                        plan->cfl_cells, plan->nlevels, plan->P, plan->d_smax,
                                        dt_dev, s);
  if (e != hipSuccess) return hip_fail(e, "cfl launch");
  return PPM_OK;
}

ppm_status sweep_checked(ppm_plan *plan, const double *dt_dev, int32_t axis, int32_t active_mask,
                         bool cfl, void *hip_stream) {
  if (!plan) return fail(PPM_EINVAL, "plan is NULL");
  if (!dt_dev) return fail(PPM_EINVAL, "dt_dev is NULL");
  if (axis < 0 || axis > 2) return fail(PPM_EINVAL, "axis must be 0, 1 or 2");
  if (active_mask < 0 || active_mask > 7) return fail(PPM_EINVAL, "active_mask must be in 0..7");
  hipError_t e = sweep_any(plan, dt_dev, axis, active_mask & ~(1 << axis),
                           cfl ? plan->d_smax : nullptr, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "sweep launch");
  return PPM_OK;
}

ppm_status step_any(ppm_plan *plan, const double *dt_dev, int32_t sweep_order, bool cfl,
                    hipStream_t s) {
  unsigned long long *smax = cfl ? plan->d_smax : nullptr;
  if (plan->persistent) {
    hipError_t e = plan->prec == PPM_FP64
        ? ppm::launch_batch<ppm::PrecF64>(plan->d_patches, plan->d_order, plan->npatch,
                                          plan->batch_blocks, plan->batch_block, sweep_order,
                                          plan->lanes_mask, dt_dev, plan->P, plan->d_counters,
                                          plan->d_queue, smax, s)
        : ppm::launch_batch<ppm::PrecMixed>(plan->d_patches, plan->d_order, plan->npatch,
                                            plan->batch_blocks, plan->batch_block, sweep_order,
                                            plan->lanes_mask, dt_dev, plan->P, plan->d_counters,
                                            plan->d_queue, smax, s);
    if (e != hipSuccess) return hip_fail(e, "persistent step launch");
    return PPM_OK;
  }
  int mask = 0;
  for (int k = 0; k < 3; ++k) {
    const int axis = kOrders[sweep_order][k];
    hipError_t e = sweep_any(plan, dt_dev, axis, mask, k == 2 ? smax : nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "sweep launch");
    mask |= 1 << axis;
  }
  return PPM_OK;
}

ppm_status ppm_sweep(ppm_plan *plan, const double *dt_dev, int32_t axis, int32_t active_mask,
                     void *hip_stream) {
  return sweep_checked(plan, dt_dev, axis, active_mask, false, hip_stream);
}

ppm_status ppm_sweep_cfl(ppm_plan *plan, const double *dt_dev, int32_t axis,
                         int32_t active_mask, void *hip_stream) {
  return sweep_checked(plan, dt_dev, axis, active_mask, true, hip_stream);
}

ppm_status ppm_cfl_finalize(ppm_plan *plan, double *dt_dev, void *hip_stream) {
  if (!plan) return fail(PPM_EINVAL, "plan is NULL");
  if (!dt_dev) return fail(PPM_EINVAL, "dt_dev is NULL");
  hipError_t e = ppm::launch_cfl_finalize(plan->nlevels, plan->P.cfl, plan->P.expand,
                                          plan->d_smax, dt_dev,
                                          static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "cfl finalize launch");
  return PPM_OK;
}

ppm_status ppm_step(ppm_plan *plan, const double *dt_dev, int32_t sweep_order,
                    void *hip_stream) {
  if (!plan) return fail(PPM_EINVAL, "plan is NULL");
  if (!dt_dev) return fail(PPM_EINVAL, "dt_dev is NULL");
  if (sweep_order < 0 || sweep_order > 5) return fail(PPM_EINVAL, "sweep_order must be in 0..5");
  return step_any(plan, dt_dev, sweep_order, false, static_cast<hipStream_t>(hip_stream));
}

ppm_status ppm_step_cfl(ppm_plan *plan, double *dt_dev, int32_t sweep_order, void *hip_stream) {
  if (!plan) return fail(PPM_EINVAL, "plan is NULL");
  if (!dt_dev) return fail(PPM_EINVAL, "dt_dev is NULL");
  if (sweep_order < 0 || sweep_order > 5) return fail(PPM_EINVAL, "sweep_order must be in 0..5");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  ppm_status st = step_any(plan, dt_dev, sweep_order, true, s);
  if (st != PPM_OK) return st;
  return ppm_cfl_finalize(plan, dt_dev, s);
}

ppm_status ppm_event_counts(ppm_plan *plan, int64_t *fallback_faces, int64_t *floored_cells,
                            int32_t reset, void *hip_stream) {
  if (!plan) return fail(PPM_EINVAL, "plan is NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  unsigned long long h[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(h, plan->d_counters, sizeof h, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "event counter read");
  if (fallback_faces) *fallback_faces = int64_t(h[0]);
  if (floored_cells) *floored_cells = int64_t(h[1]);
  if (reset) {
    static const unsigned long long z[2] = {0, 0};
    e = hipMemcpyAsync(plan->d_counters, z, sizeof z, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "event counter reset");
  }
  return PPM_OK;
}

struct ppm_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

ppm_status ppm_graph_create(ppm_graph **out, ppm_plan *plan, double *dt_dev,
                            int32_t sweep_order, uint32_t parts, void *hip_stream) {
  (void)hip_stream;
  if (!out) return fail(PPM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!plan) return fail(PPM_EINVAL, "plan is NULL");
  if (!dt_dev) return fail(PPM_EINVAL, "dt_dev is NULL");
  if (parts == 0 || (parts & ~15u))
    return fail(PPM_EINVAL, "parts must be a non-empty subset of FILL|CFL|STEP|STEP_CFL");
  if ((parts & PPM_GRAPH_STEP) && (parts & PPM_GRAPH_STEP_CFL))
    return fail(PPM_EINVAL, "parts: STEP and STEP_CFL exclude each other");
  if ((parts & (PPM_GRAPH_STEP | PPM_GRAPH_STEP_CFL)) && (sweep_order < 0 || sweep_order > 5))
    return fail(PPM_EINVAL, "sweep_order must be in 0..5");
  ppm_graph *g = new (std::nothrow) ppm_graph();
  if (!g) return fail(PPM_ENOMEM, "host allocation failed");
  hipStream_t cs = nullptr;  // capture on a private stream (the null stream cannot be captured)
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "capture stream");
  }
  ppm_status st = PPM_OK;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    if (parts & PPM_GRAPH_FILL) st = ppm_fill_periodic(plan, cs);
    if (st == PPM_OK && (parts & PPM_GRAPH_CFL)) st = ppm_cfl_dt(plan, dt_dev, cs);
    if (st == PPM_OK && (parts & PPM_GRAPH_STEP)) st = ppm_step(plan, dt_dev, sweep_order, cs);
    if (st == PPM_OK && (parts & PPM_GRAPH_STEP_CFL))
      st = ppm_step_cfl(plan, dt_dev, sweep_order, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
    if (st == PPM_OK && e2 != hipSuccess) st = hip_fail(e2, "end capture");
    if (st == PPM_OK) {
      e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) st = hip_fail(e, "graph instantiate");
    }
  } else {
    st = hip_fail(e, "begin capture");
  }
  (void)hipStreamDestroy(cs);
  if (st != PPM_OK) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return st;
  }
  *out = g;
  return PPM_OK;
}

ppm_status ppm_graph_launch(ppm_graph *graph, void *hip_stream) {
  if (!graph || !graph->exec) return fail(PPM_EINVAL, "graph is NULL");
  hipError_t e = hipGraphLaunch(graph->exec, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  return PPM_OK;
}

ppm_status ppm_graph_destroy(ppm_graph *graph) {
  if (!graph) return PPM_OK;
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  delete graph;
  return PPM_OK;
}

const char *ppm_status_str(ppm_status st) {
  switch (st) {
    case PPM_OK: return "PPM_OK";
    case PPM_EINVAL: return "PPM_EINVAL: invalid argument";
    case PPM_ENOMEM: return "PPM_ENOMEM: allocation failed";
    case PPM_EHIP: return "PPM_EHIP: HIP runtime error";
    case PPM_EUNSUPPORTED: return "PPM_EUNSUPPORTED: not supported";
  }
  return "unknown ppm_status";
}

const char *ppm_last_error(void) { return ppm_detail::g_last_error.c_str(); }

}  // extern "C"
