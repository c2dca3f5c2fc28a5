// ppm_noalloc.cpp -- ppm_step_cfl_noalloc: a step of up to
// PPM_NOALLOC_MAX_PATCHES patches that allocates nothing.
//
// A plan owns device memory for its patch table, launch maps, event
// counters and per-level CFL maxima.  This entry point keeps the same four
// in `scratch`, a static device array of PPM_NOALLOC_SCRATCH_BYTES bytes that
// every device the library runs on holds until the process ends: the host
// computes the table and the maps on the stack, writes them into the array
// with small kernels that take them as arguments (no staging copy, no
// memset), and launches the plan's own sweep, CFL and fill kernels on
// pointers into it.  The array's device address is taken once per device
// (hipGetSymbolAddress, with that device current) and kept; the name
// `scratch` itself is a host-side stand-in and is never passed anywhere.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>

#include "ppm.h"
#include "ppm_kernels.hpp"
#include "ppm_plan.hpp"

using ppm_detail::fail;
using ppm_detail::hip_fail;

namespace {

constexpr int kMaxPatches = PPM_NOALLOC_MAX_PATCHES;
constexpr int kMaxLevels = PPM_NOALLOC_MAX_PATCHES;
constexpr int kMaxDevices = 64;
constexpr int kSlots = 25;  // 12 marching and 12 lane-parallel sweep maps, then the CFL map
constexpr int kStride = kMaxPatches + 1;
constexpr int kCflCells = 4096;

// Layout of the scratch array.
constexpr size_t kPatchOff = 0;
constexpr size_t kChunkOff = kPatchOff + sizeof(PatchDev) * kMaxPatches;
constexpr size_t kCountOff = (kChunkOff + sizeof(int32_t) * kSlots * kStride + 255) / 256 * 256;
constexpr size_t kSmaxOff = kCountOff + 2 * sizeof(unsigned long long);
constexpr size_t kUsedBytes = kSmaxOff + kMaxLevels * sizeof(unsigned long long);
static_assert(kUsedBytes <= PPM_NOALLOC_SCRATCH_BYTES, "scratch layout exceeds its size");
static_assert(kChunkOff % 8 == 0 && kCountOff % 8 == 0, "alignment");

const int kOrders[6][3] = {{0, 1, 2}, {2, 1, 0}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}};

}  // namespace

static __device__ __align__(256) unsigned char scratch[PPM_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
unsigned char *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (taken once per device).
ppm_status scratch_address(unsigned char **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(PPM_EUNSUPPORTED, "device %d: at most %d devices are supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = static_cast<unsigned char *>(p);
  }
  *out = g_scratch[dev];
  return PPM_OK;
}

inline int t1_of(int axis) { return axis == 0 ? 1 : 0; }
inline int t2_of(int axis) { return axis == 2 ? 1 : 2; }

// Launch shapes of the call: as a plan over the same patches with the
// default tile configuration, per-sweep launches (no persistent launch, no
// grouped maps: each block belongs to one patch).
struct Shapes {
  int32_t block, lanes_block;
  int32_t nblocks[kSlots];
  int32_t tail_pencil0[2][12], tail_main[2][12], tail_blocks[2][12];
};

template <class Prec>
hipError_t sweep(const Shapes &sh, const PatchDev *patches, const int32_t *chunks, int npatch,
                 int axis, int mask, const double *dt, const ppm::Params &P,
                 unsigned long long *counters, unsigned long long *smax, hipStream_t s) {
  const int tm = ((mask >> t1_of(axis)) & 1) | (((mask >> t2_of(axis)) & 1) << 1);
  if (axis == 0) {  // x sweeps: cells across the lanes
    const int slot = 12 + tm;
    if (sh.nblocks[slot] == 0) return hipSuccess;
    return ppm::launch_sweep_lanes<Prec>(patches, chunks + slot * kStride, npatch,
                                         sh.nblocks[slot], sh.lanes_block, axis, mask, dt, P,
                                         counters, smax, s);
  }
  const int slot = axis * 4 + tm, c = smax ? 1 : 0;
  const int32_t *cs = chunks + slot * kStride;
  if (sh.nblocks[slot] == 0) return hipSuccess;
  if (sh.tail_blocks[c][slot] > 0) {
    hipError_t e = ppm::launch_sweep<Prec>(patches, cs, npatch, sh.tail_main[c][slot], sh.block,
                                           axis, mask, dt, P, counters, smax, nullptr, 0, s);
    if (e != hipSuccess) return e;
    return ppm::launch_sweep_tail<Prec>(patches, cs, sh.tail_blocks[c][slot], sh.lanes_block,
                                        axis, mask, sh.tail_pencil0[c][slot], dt, P, counters,
                                        smax, s);
  }
  return ppm::launch_sweep<Prec>(patches, cs, npatch, sh.nblocks[slot], sh.block, axis, mask, dt,
                                 P, counters, smax, nullptr, 0, s);
}

template <class Prec>
hipError_t run(const Shapes &sh, const PatchDev *host, const int32_t *bc, unsigned char *base,
               int npatch,
               int nlevels, const ppm::Params &P, double *dt, int sweep_order, uint32_t parts,
               int32_t cfl_blocks, hipStream_t s) {
  const PatchDev *patches = reinterpret_cast<const PatchDev *>(base + kPatchOff);
  const int32_t *chunks = reinterpret_cast<const int32_t *>(base + kChunkOff);
  unsigned long long *counters = reinterpret_cast<unsigned long long *>(base + kCountOff);
  unsigned long long *smax = reinterpret_cast<unsigned long long *>(base + kSmaxOff);
  hipError_t e = hipSuccess;
  if (parts & PPM_NOALLOC_FILL)
    for (int i = 0; i < npatch && e == hipSuccess; ++i)
      if (bc[i] == PPM_BC_PERIODIC) e = ppm::launch_fill<Prec>(host[i], s);
  if (e == hipSuccess && (parts & PPM_NOALLOC_CFL))
    e = ppm::launch_cfl<Prec>(patches, chunks + 24 * kStride, npatch, cfl_blocks, kCflCells,
                              nlevels, P, smax, dt, s);
  int mask = 0;
  for (int k = 0; k < 3 && e == hipSuccess; ++k) {
    const int axis = kOrders[sweep_order][k];
    e = sweep<Prec>(sh, patches, chunks, npatch, axis, mask, dt, P, counters,
                    k == 2 ? smax : nullptr, s);
    mask |= 1 << axis;
  }
  if (e == hipSuccess) e = ppm::launch_cfl_finalize(nlevels, P.cfl, nullptr, smax, dt, s);
  return e;
}

}  // namespace

extern "C" ppm_status ppm_step_cfl_noalloc(const ppm_patch *patches, int32_t npatch,
                                           int32_t nlevels, ppm_precision prec,
                                           const ppm_params *params, double *dt_dev,
                                           int32_t sweep_order, uint32_t parts, int64_t *events,
                                           void *hip_stream) {
  if (!patches) return fail(PPM_EINVAL, "patches is NULL");
  if (npatch < 1 || npatch > kMaxPatches)
    return fail(PPM_EINVAL, "npatch must be in 1..%d (the static scratch holds %d patches)",
                kMaxPatches, kMaxPatches);
  if (nlevels < 1 || nlevels > kMaxLevels)
    return fail(PPM_EINVAL, "nlevels must be in 1..%d (the static scratch holds %d levels)",
                kMaxLevels, kMaxLevels);
  if (prec != PPM_FP64 && prec != PPM_MIXED) return fail(PPM_EINVAL, "unknown precision %d", int(prec));
  if (!dt_dev) return fail(PPM_EINVAL, "dt_dev is NULL");
  if (sweep_order < 0 || sweep_order > 5) return fail(PPM_EINVAL, "sweep_order must be in 0..5");
  if (parts & ~uint32_t(PPM_NOALLOC_FILL | PPM_NOALLOC_CFL))
    return fail(PPM_EINVAL, "unknown parts bits 0x%x", parts);
  ppm_status st = ppm_detail::check_params(params);
  if (st != PPM_OK) return st;
  if ((st = ppm_detail::check_mixed_floors(prec, params)) != PPM_OK) return st;
  for (int i = 0; i < npatch; ++i)
    if ((st = ppm_detail::check_patch(patches[i], i, nlevels)) != PPM_OK) return st;
  ppm::Params P = ppm_detail::device_params(prec, params);

  // patch table
  PatchDev host[kMaxPatches];
  int32_t bc[kMaxPatches] = {};
  std::memset(host, 0, sizeof host);
  for (int i = 0; i < npatch; ++i) {
    const ppm_patch &q = patches[i];
    PatchDev &d = host[i];
    d.n[0] = q.nx; d.n[1] = q.ny; d.n[2] = q.nz;
    d.ghost = q.ghost; d.level = q.level; d.pad = 0;
    bc[i] = q.bc;
    d.dx[0] = q.dx; d.dx[1] = q.dy; d.dx[2] = q.dz;
    d.rho = q.rho; d.vel[0] = q.vx; d.vel[1] = q.vy; d.vel[2] = q.vz;
    d.etot = q.etot; d.eint = q.eint; d.flux_reg = q.flux_reg;
    d.acc[0] = q.gx; d.acc[1] = q.gy; d.acc[2] = q.gz;
    if (q.gx) P.flags |= ppm::kAnyGravity;
  }
  if ((parts & PPM_NOALLOC_FILL))
    for (int i = 0; i < npatch; ++i)
      if (patches[i].bc != PPM_BC_PERIODIC)
        return fail(PPM_EINVAL, "patch %d: PPM_NOALLOC_FILL needs PPM_BC_PERIODIC patches", i);

  // launch maps (prefix arrays of work chunks per sweep slot, then the CFL map)
  Shapes sh;
  std::memset(&sh, 0, sizeof sh);
  sh.block = npatch == 1 ? 256 : 64;
  sh.lanes_block = npatch == 1 ? 256 : 64;
  int32_t chunks[kSlots * kStride];
  std::memset(chunks, 0, sizeof chunks);
  for (int kind = 0; kind < 2; ++kind)
    for (int axis = 0; axis < 3; ++axis)
      for (int tm = 0; tm < 4; ++tm) {
        const int slot = kind * 12 + axis * 4 + tm;
        int64_t acc = 0;
        for (int i = 0; i < npatch; ++i) {
          const PatchDev &d = host[i];
          const int64_t w1 = (tm & 1) ? d.n[t1_of(axis)] : d.n[t1_of(axis)] + 2 * d.ghost;
          const int64_t w2 = (tm & 2) ? d.n[t2_of(axis)] : d.n[t2_of(axis)] + 2 * d.ghost;
          int64_t items = w1 * w2, per_block = sh.block;
          if (kind == 1) {
            const int64_t rpw = ppm::rows_per_wave(int(d.n[axis] + 2 * d.ghost));
            items = (items + rpw - 1) / rpw;
            per_block = sh.lanes_block / 64;
          }
          chunks[slot * kStride + i] = int32_t(acc);
          acc += (items + per_block - 1) / per_block;
          if (acc > INT32_MAX / 2) return fail(PPM_EINVAL, "too many pencils for one launch");
        }
        chunks[slot * kStride + npatch] = int32_t(acc);
        sh.nblocks[slot] = int32_t(acc);
      }
  int32_t cfl_blocks = 0;
  {
    int64_t acc = 0;
    for (int i = 0; i < npatch; ++i) {
      const PatchDev &d = host[i];
      chunks[24 * kStride + i] = int32_t(acc);
      acc += (int64_t(d.n[0]) * d.n[1] * d.n[2] + kCflCells - 1) / kCflCells;
      if (acc > INT32_MAX / 2) return fail(PPM_EINVAL, "too many cells for one CFL launch");
    }
    chunks[24 * kStride + npatch] = int32_t(acc);
    cfl_blocks = int32_t(acc);
  }
  // one patch: whole rounds of one marching block per compute unit, the few
  // pencils left over to the lane-parallel tail launch (as a one-patch plan
  // does)
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 0;
  if (npatch == 1 && cus > 0)
    for (int c = 0; c < 2; ++c) {
      const int64_t cap = int64_t(cus) * sh.block;
      if (cap <= 0) continue;
      for (int slot = 0; slot < 12; ++slot) {
        const int axis = slot / 4, tm = slot % 4;
        const PatchDev &d = host[0];
        const int64_t w1 = (tm & 1) ? d.n[t1_of(axis)] : d.n[t1_of(axis)] + 2 * d.ghost;
        const int64_t w2 = (tm & 2) ? d.n[t2_of(axis)] : d.n[t2_of(axis)] + 2 * d.ghost;
        const int64_t np = w1 * w2, rest = np % cap;
        if (np < cap || rest == 0 || rest * 8 > cap) continue;
        sh.tail_pencil0[c][slot] = int32_t(np - rest);
        sh.tail_main[c][slot] = int32_t((np - rest) / sh.block);
        sh.tail_blocks[c][slot] = int32_t((rest + sh.lanes_block / 64 - 1) / (sh.lanes_block / 64));
      }
    }

  unsigned char *base = nullptr;
  if ((st = scratch_address(&base)) != PPM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // the table, the maps, and zeroed counters and maxima (the previous call's
  // contents are all replaced)
  uint32_t words[kUsedBytes / 4];
  std::memset(words, 0, sizeof words);
  std::memcpy(reinterpret_cast<unsigned char *>(words) + kPatchOff, host, sizeof host);
  std::memcpy(reinterpret_cast<unsigned char *>(words) + kChunkOff, chunks, sizeof chunks);
  hipError_t e = ppm::launch_write_words(reinterpret_cast<uint32_t *>(base), words,
                                         int64_t(kUsedBytes / 4), s);
  if (e != hipSuccess) return hip_fail(e, "scratch upload");
  e = prec == PPM_FP64
          ? run<ppm::PrecF64>(sh, host, bc, base, npatch, nlevels, P, dt_dev, sweep_order,
                              parts, cfl_blocks, s)
          : run<ppm::PrecMixed>(sh, host, bc, base, npatch, nlevels, P, dt_dev, sweep_order,
                                parts, cfl_blocks, s);
  if (e != hipSuccess) return hip_fail(e, "ppm_step_cfl_noalloc launch");
  if (events) {
    unsigned long long h[2] = {0, 0};
    e = hipMemcpyAsync(h, base + kCountOff, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "event counter read");
    events[0] = int64_t(h[0]);
    events[1] = int64_t(h[1]);
  }
  return PPM_OK;
}
