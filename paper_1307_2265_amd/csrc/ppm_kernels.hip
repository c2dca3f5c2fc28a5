// ppm_kernels.hip -- HIP kernels of the PPM library for gfx950.
//
//   * sweep_kernel: one 1-D PPM sweep over a set of patches.  The grid is a
//     flat list of (patch, chunk of pencils) work items: block b finds its
//     patch by binary search in a prefix array of chunk counts, and each
//     thread of the block marches one pencil (ppm_sweep.hpp).  A single big
//     grid is the one-patch case of the same kernel.
//   * sweep_split_kernel: the marching sweep of one patch with two threads
//     per pencil, when the pencils are too few to fill the device.
//   * sweep_lanes_kernel: the same sweep with the cells of a pencil across
//     the lanes of a wave (ppm_lanes.hpp), for x sweeps.
//   * sweep_tail_kernel: the same lane-parallel code over the last pencils of
//     a big patch's marching sweep, one pencil per wave, after the marching
//     launch has taken whole rounds of one block per compute unit.
//   * batch_persistent_kernel: a whole step of every patch in one launch.
//   * Each sweep kernel has a variant for the last sweep of a step that also
//     takes the max signal speed of the cells it writes, so the next step's
//     timestep needs no pass of its own (cfl_finalize_kernel turns the max
//     into dt).
//   * cfl_reduce_kernel / cfl_finalize_kernel: the hydro CFL timestep of
//     every level (Sec. "Timestepping"): a wave-level max of the per-cell
//     signal speed sum_d (c_s + |v_d|)/dx_d, a block max through LDS, and a
//     device-wide max by atomicMax on the bit pattern of the non-negative
//     double; the finalise kernel turns the max into dt and clears it.
//   * fill_periodic_kernel: periodic ghost fill of one patch over its ghost
//     shell only; fill_boundary_kernel: the same shell by per-face domain
//     boundary conditions; fill_from_parent_kernel / copy_from_siblings_kernel:
//     AMR patch ghosts from the parent (SecondOrderA) and from siblings.
//
// The file is compiled in four passes, each with the instruction scheduling
// under which its sweeps run fastest (see build.py): PPM_KERNEL_PASS 1 emits
// the double-precision marching sweeps and every non-sweep kernel, 2 the
// mixed-precision marching sweeps, 3 the double-precision lane-parallel
// sweeps (lanes and tail), 4 the mixed-precision lane-parallel ones; without
// the macro one pass emits everything.
#include "ppm_kernels.hpp"
#include "ppm_lanes.hpp"

#ifndef PPM_KERNEL_PASS
#define PPM_KERNEL_PASS 0
#endif
#define PPM_PASS_FP64 (PPM_KERNEL_PASS == 0 || PPM_KERNEL_PASS == 1)
#define PPM_PASS_MIXED (PPM_KERNEL_PASS == 0 || PPM_KERNEL_PASS == 2)
#define PPM_PASS_FP64_LANES (PPM_KERNEL_PASS == 0 || PPM_KERNEL_PASS == 3)
#define PPM_PASS_MIXED_LANES (PPM_KERNEL_PASS == 0 || PPM_KERNEL_PASS == 4)

namespace ppm {

__device__ __forceinline__ int find_patch(const int32_t *start, int32_t npatch, int32_t b) {
  int lo = 0, hi = npatch - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Fold a wave's signal-speed maxima into the level's device-wide max: a
// wave-level max, then atomicMax on the bit pattern of the non-negative
// double (which orders like the value).
__device__ __forceinline__ void cfl_commit(double smax, unsigned long long *slot) {
  smax = wave_max(smax);
  if ((threadIdx.x & 63) == 0 && smax > 0.0)
    atomicMax(slot, (unsigned long long)__double_as_longlong(smax));
}

// Largest i in [lo, hi) with a[i] <= x (a non-decreasing, a[lo] <= x).
__device__ __forceinline__ int last_at_most(const int32_t *a, int lo, int hi, int32_t x) {
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Fold each lane's signal-speed maximum into its own level's maximum, for
// waves whose lanes may belong to patches of different levels.
__device__ __forceinline__ void cfl_commit_levels(double smax, int level,
                                                  unsigned long long *smax_bits) {
  const int lane = threadIdx.x & 63;
  unsigned long long pending = __ballot(smax > 0.0);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int L = __shfl(level, leader, 64);
    const bool take = smax > 0.0 && level == L;
    const double m = wave_max(take ? smax : 0.0);
    if (lane == leader) atomicMax(&smax_bits[L], (unsigned long long)__double_as_longlong(m));
    pending &= ~__ballot(take);
  }
}

// One thread marches one pencil.  Ungrouped: each block takes `blockDim.x`
// consecutive pencils of one patch (block -> patch by the prefix array
// chunk_start).  Grouped (several patches): patches are sorted by pencil
// length (longest first) and the pencils of a run of equal-length patches are numbered
// consecutively, so a block's threads may belong to several patches and no
// wave is left partly empty at a patch's end; `groups` holds, for this
// sweep, the first block and the first sorted patch of every run, the
// pencil prefix over the sorted patches, and the sorted patch indices.  The
// patches of a run are views into six shared arrays at one element offset
// per patch, so the field pointers of the run's first patch serve the whole
// wave and only the offset, strides and cell width vary per lane.
template <class Prec, bool kCFL, bool kGrouped, bool kUseHLLC, bool kGrav>
__global__ void __launch_bounds__(kMaxBlock, 2)
sweep_kernel(const PatchDev *__restrict__ patches, const int32_t *__restrict__ chunk_start,
             int32_t npatch, int32_t axis, int32_t mask, const double *__restrict__ dt_dev,
             Params P, unsigned long long *__restrict__ counters,
             unsigned long long *__restrict__ smax_bits, const int32_t *__restrict__ groups,
             int32_t ngroups) {
  using S = typename Prec::S;
  extern __shared__ double lds[];
  int p, idx, pref = 0;
  bool has;
  if (kGrouped) {
    const int32_t *gbs = groups, *gfirst = groups + ngroups + 1;
    const int32_t *pp = gfirst + ngroups + 1, *sorted = pp + npatch + 1;
    const int grp = last_at_most(gbs, 0, ngroups, int32_t(blockIdx.x));
    const int j0 = gfirst[grp], j1 = gfirst[grp + 1];
    const int q = pp[j0] + (int(blockIdx.x) - gbs[grp]) * int(blockDim.x) + int(threadIdx.x);
    has = q < pp[j1];
    const int j = has ? last_at_most(pp, j0, j1, q) : j0;
    p = sorted[j];
    pref = sorted[j0];
    idx = has ? q - pp[j] : 0;
  } else {
    p = find_patch(chunk_start, npatch, blockIdx.x);
    idx = (blockIdx.x - chunk_start[p]) * blockDim.x + threadIdx.x;
    has = true;
  }
  const PatchDev pd = patches[p];
  int i1 = pd.ghost, i2 = pd.ghost;
  has = has && pencil_index(pd, axis, mask, idx, i1, i2);
  if (!kCFL && !has) return;
  CflAcc cfl = cfl_acc(pd, axis, lds + kLdsCfl * int(blockDim.x) + threadIdx.x);
  if (kCFL) *cfl.lds = 0.0;
  uint32_t nfb = 0, nfl = 0;
  if (has) {
    PencilRef<S> pc = make_pencil<S>(pd, axis, i1, i2);
    if (kGrouped) {
      // equal within a run of patches: keep the loop bounds scalar; address
      // through the (wave-uniform) field pointers of the run's first patch
      pc.n = __builtin_amdgcn_readfirstlane(pc.n);
      pc.g = __builtin_amdgcn_readfirstlane(pc.g);
      const PencilRef<S> ref = make_pencil<S>(patches[__builtin_amdgcn_readfirstlane(pref)],
                                              axis, 0, 0);
      pc.base += pc.rho - ref.rho;
      pc.rho = ref.rho; pc.u = ref.u; pc.v1 = ref.v1; pc.v2 = ref.v2; pc.E = ref.E; pc.e = ref.e;
      pc.acc = ref.acc;
    }
    const double dt = dt_dev[pd.level];
    march_pencil<Prec, kCFL, kUseHLLC, kGrav>(P, pc, dt, expansion_a(P, pd.level),
                                              lds + threadIdx.x, blockDim.x, nfb, nfl, cfl);
  }
  if (nfb) atomicAdd(&counters[0], (unsigned long long)nfb);
  if (nfl) atomicAdd(&counters[1], (unsigned long long)nfl);
  if (kCFL) {  // every lane of the wave takes part
    if (kGrouped) cfl_commit_levels(*cfl.lds, pd.level, smax_bits);
    else cfl_commit(*cfl.lds, &smax_bits[pd.level]);
  }
}

// The marching sweep of one patch with two threads per pencil, for sweeps
// with too few pencils to give every SIMD two waves: lanes 0-31 of a wave
// march the first halves of 32 consecutive pencils and lanes 32-63 the second
// halves, from max(5, g) cells before their first own cell (see MarchSpan).
// The second half stores its first five cells only after its march, from
// `defer` (30 doubles per pencil): the first half reads them as input at the
// end of its own march, and the wave leaves the march loop only when both
// halves have finished it.
template <class Prec, bool kCFL, bool kUseHLLC, bool kGrav>
__global__ void __launch_bounds__(kMaxBlock, 2)
sweep_split_kernel(const PatchDev *__restrict__ patches, int32_t axis, int32_t mask,
                   const double *__restrict__ dt_dev, Params P,
                   unsigned long long *__restrict__ counters,
                   unsigned long long *__restrict__ smax_bits, double *__restrict__ defer) {
  using S = typename Prec::S;
  extern __shared__ double lds[];
  const int t = int(blockIdx.x * blockDim.x + threadIdx.x);
  const int half = (t >> 5) & 1;
  const int idx = (t >> 6) * 32 + (t & 31);
  const PatchDev pd = patches[0];
  int i1 = pd.ghost, i2 = pd.ghost;
  const bool has = pencil_index(pd, axis, mask, idx, i1, i2);
  if (!kCFL && !has) return;
  CflAcc cfl = cfl_acc(pd, axis, lds + kLdsCfl * int(blockDim.x) + threadIdx.x);
  if (kCFL) *cfl.lds = 0.0;
  uint32_t nfb = 0, nfl = 0;
  if (has) {
    const PencilRef<S> pc = make_pencil<S>(pd, axis, i1, i2);
    const double dt = dt_dev[pd.level];
    const int g = pc.g, a1 = pc.n - g - 1;
    const int m = g + (pc.n - 2 * g + 1) / 2;  // first cell of the second half
    double *mine = defer + int64_t(idx) * (kDeferCells * 6);
    // the second half starts at least five cells, and at least g, before its
    // first own cell (its first g cells are its ghosts)
    const int lead = g > kDeferCells ? g : kDeferCells;
    const MarchSpan span = half ? MarchSpan{m - lead, pc.n - g + 4, m, a1, m, mine}
                                : MarchSpan{0, m + 4, g, m - 1, 0, nullptr};
    march_pencil<Prec, kCFL, kUseHLLC, kGrav>(P, pc, dt, expansion_a(P, pd.level),
                                              lds + threadIdx.x, blockDim.x, nfb, nfl, cfl, &span);
    if (half) {
      for (int c = 0; c < kDeferCells; ++c) {
        const int64_t o = pc.base + int64_t(m + c) * pc.stride;
        const double *d = mine + c * 6;
        pc.rho[o] = S(d[0]);
        pc.u[o] = S(d[1]);
        pc.v1[o] = S(d[2]);
        pc.v2[o] = S(d[3]);
        pc.E[o] = d[4];
        pc.e[o] = d[5];
      }
    }
  }
  if (nfb) atomicAdd(&counters[0], (unsigned long long)nfb);
  if (nfl) atomicAdd(&counters[1], (unsigned long long)nfl);
  if (kCFL) cfl_commit(*cfl.lds, &smax_bits[pd.level]);  // every lane of the wave takes part
}

// One wavefront streams a run of `rows` consecutive pencils (rows_per_wave(n)
// if rows is 0) with the cells across its lanes, from pencil `pencil0` of the
// patch on.
template <class Prec, bool kCFL, bool kUseHLLC, bool kGrav>
__device__ __forceinline__ void stream_pencils(const PatchDev *__restrict__ patches,
                                               const int32_t *__restrict__ chunk_start,
                                               int32_t npatch, int32_t axis, int32_t mask,
                                               int32_t pencil0, int32_t rows,
                                               const double *__restrict__ dt_dev, const Params &P,
                                               unsigned long long *__restrict__ counters,
                                               unsigned long long *__restrict__ smax_bits) {
  const int p = find_patch(chunk_start, npatch, blockIdx.x);
  const PatchDev pd = patches[p];
  const int waves = blockDim.x >> 6;
  const int item = (blockIdx.x - chunk_start[p]) * waves + (threadIdx.x >> 6);
  const int n = pick3(axis, pd.n[0], pd.n[1], pd.n[2]) + 2 * pd.ghost;
  const int K = rows > 0 ? rows : rows_per_wave(n);
  const int np = pencil_count(pd, axis, mask);
  const int first = pencil0 + item * K;
  if (first >= np) return;  // the whole wave leaves
  const double dt = dt_dev[pd.level];
  uint32_t nfb = 0, nfl = 0;
  CflAcc cfl = cfl_acc(pd, axis, nullptr);
  sweep_rows_lanes<Prec, kCFL, kUseHLLC, kGrav>(P, pd, axis, mask, first, min(K, np - first),
                                                dt, expansion_a(P, pd.level), nfb, nfl, cfl);
  if (nfb) atomicAdd(&counters[0], (unsigned long long)nfb);
  if (nfl) atomicAdd(&counters[1], (unsigned long long)nfl);
  if (kCFL) cfl_commit(cfl.smax, &smax_bits[pd.level]);
}

// Lane-parallel sweep: each wavefront streams rows_per_wave(n) pencils.
template <class Prec, bool kCFL, bool kUseHLLC, bool kGrav>
__global__ void __launch_bounds__(kMaxBlock, 4)
sweep_lanes_kernel(const PatchDev *__restrict__ patches, const int32_t *__restrict__ chunk_start,
                   int32_t npatch, int32_t axis, int32_t mask, const double *__restrict__ dt_dev,
                   Params P, unsigned long long *__restrict__ counters,
                   unsigned long long *__restrict__ smax_bits) {
  stream_pencils<Prec, kCFL, kUseHLLC, kGrav>(patches, chunk_start, npatch, axis, mask, 0, 0,
                                              dt_dev, P, counters, smax_bits);
}

// The pencils of one patch from `pencil0` on, one per wavefront: what is
// left of a marching sweep after whole rounds of one block per compute unit.
template <class Prec, bool kCFL, bool kUseHLLC, bool kGrav>
__global__ void __launch_bounds__(kMaxBlock, 4)
sweep_tail_kernel(const PatchDev *__restrict__ patches, const int32_t *__restrict__ chunk_start,
                  int32_t axis, int32_t mask, int32_t pencil0, const double *__restrict__ dt_dev,
                  Params P, unsigned long long *__restrict__ counters,
                  unsigned long long *__restrict__ smax_bits) {
  stream_pencils<Prec, kCFL, kUseHLLC, kGrav>(patches, chunk_start, 1, axis, mask, pencil0, 1,
                                              dt_dev, P, counters, smax_bits);
}

// ---------------------------------------------------------------------------
// Persistent batch kernel: one launch advances every patch by a full step.
// Workgroups take patches from a queue (an atomic counter over the patches
// in descending order of cost) and run the three sweeps of each patch one
// after the other, separated by workgroup barriers; the workgroup's threads
// share the pencils of each sweep (sweeps along the lane-parallel axes are
// streamed by the waves, the rest marched by the threads).  No
// workgroup ever waits for another, and every workgroup leaves once the queue
// is empty; the last one to leave rewinds the queue for the next launch.

__constant__ int kStepOrders[6][3] = {{0, 1, 2}, {2, 1, 0}, {0, 2, 1},
                                      {1, 0, 2}, {1, 2, 0}, {2, 0, 1}};

template <class Prec, bool kCFL, bool kUseHLLC, bool kGrav>
__global__ void __launch_bounds__(kMaxBlock, 2)
batch_persistent_kernel(const PatchDev *__restrict__ patches, const int32_t *__restrict__ order,
                        int32_t npatch, int32_t sweep_order, int32_t lanes_mask,
                        const double *__restrict__ dt_dev, Params P,
                        unsigned long long *__restrict__ counters, unsigned int *queue,
                        unsigned long long *__restrict__ smax_bits) {
  using S = typename Prec::S;
  extern __shared__ double lds[];
  __shared__ int s_item;
  uint32_t nfb = 0, nfl = 0;
  const int wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  for (;;) {
    if (threadIdx.x == 0) s_item = int(atomicAdd(&queue[0], 1u));
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= npatch) break;
    const PatchDev pd = patches[order[item]];
    const double dt = dt_dev[pd.level];
    int mask = 0;
    for (int k = 0; k < 3; ++k) {
      const int axis = kStepOrders[sweep_order][k];
      const int t1 = axis == 0 ? 1 : 0, t2 = axis == 2 ? 1 : 2;
      const int g = pd.ghost;
      const int Nt1 = pick3(t1, pd.n[0], pd.n[1], pd.n[2]);
      const int Nt2 = pick3(t2, pd.n[0], pd.n[1], pd.n[2]);
      const int w1 = ((mask >> t1) & 1) ? Nt1 : Nt1 + 2 * g;
      const int w2 = ((mask >> t2) & 1) ? Nt2 : Nt2 + 2 * g;
      const int np = w1 * w2;
      const int n = pick3(axis, pd.n[0], pd.n[1], pd.n[2]) + 2 * g;
      int i1, i2;
      CflAcc cfl = cfl_acc(pd, axis, lds + kLdsCfl * int(blockDim.x) + threadIdx.x);
      if (kCFL && k == 2) *cfl.lds = 0.0;
      if ((lanes_mask >> axis) & 1) {
        const int K = rows_per_wave(n);
        for (int first = wave * K; first < np; first += waves * K) {
          if (kCFL && k == 2)
            sweep_rows_lanes<Prec, true, kUseHLLC, kGrav>(P, pd, axis, mask, first,
                                                          min(K, np - first), dt,
                                                          expansion_a(P, pd.level), nfb, nfl,
                                                          cfl);
          else
            sweep_rows_lanes<Prec, false, kUseHLLC, kGrav>(P, pd, axis, mask, first,
                                                           min(K, np - first), dt,
                                                           expansion_a(P, pd.level), nfb, nfl,
                                                           cfl);
        }
      } else {
        for (int idx = threadIdx.x; idx < np; idx += blockDim.x) {
          pencil_index(pd, axis, mask, idx, i1, i2);
          const PencilRef<S> pc = make_pencil<S>(pd, axis, i1, i2);
          if (kCFL && k == 2)
            march_pencil<Prec, true, kUseHLLC, kGrav>(P, pc, dt, expansion_a(P, pd.level),
                                                      lds + threadIdx.x, blockDim.x, nfb, nfl,
                                                      cfl);
          else
            march_pencil<Prec, false, kUseHLLC, kGrav>(P, pc, dt, expansion_a(P, pd.level),
                                                       lds + threadIdx.x, blockDim.x, nfb, nfl,
                                                       cfl);
        }
      }
      if (kCFL && k == 2)
        cfl_commit(((lanes_mask >> axis) & 1) ? cfl.smax : *cfl.lds, &smax_bits[pd.level]);
      __syncthreads();  // this sweep of the patch is complete before the next reads it
      mask |= 1 << axis;
    }
  }
  if (nfb) atomicAdd(&counters[0], (unsigned long long)nfb);
  if (nfl) atomicAdd(&counters[1], (unsigned long long)nfl);
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&queue[1], 1u) == gridDim.x - 1) {  // last workgroup out
      atomicExch(&queue[0], 0u);
      atomicExch(&queue[1], 0u);
    }
  }
}

#if PPM_PASS_FP64
// ---------------------------------------------------------------------------
// CFL reduction

template <class Prec>
__global__ void __launch_bounds__(256)
cfl_reduce_kernel(const PatchDev *__restrict__ patches, const int32_t *__restrict__ chunk_start,
                  int32_t npatch, int32_t cells_per_block, Params P,
                  unsigned long long *__restrict__ smax_bits) {
  using S = typename Prec::S;
  __shared__ double wmax[kMaxBlock / 64];
  const int p = find_patch(chunk_start, npatch, blockIdx.x);
  const PatchDev pd = patches[p];
  const int g = pd.ghost;
  const int64_t nx = pd.n[0], ny = pd.n[1];
  const int64_t total = nx * ny * pd.n[2];
  const int64_t nfx = nx + 2 * g, nfy = ny + 2 * g;
  const int64_t c0 = int64_t(blockIdx.x - chunk_start[p]) * cells_per_block;
  const int64_t c1 = c0 + cells_per_block < total ? c0 + cells_per_block : total;
  const S *rho = static_cast<const S *>(pd.rho);
  const S *vx = static_cast<const S *>(pd.vel[0]);
  const S *vy = static_cast<const S *>(pd.vel[1]);
  const S *vz = static_cast<const S *>(pd.vel[2]);
  double smax = 0.0;
  for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
    const int64_t x = c % nx, yz = c / nx;
    const int64_t y = yz % ny, z = yz / ny;
    const int64_t o = ((z + g) * nfy + (y + g)) * nfx + (x + g);
    const double s = cell_signal<S>(P, 0, pd.dx, rho[o], vx[o], vy[o], vz[o], pd.etot[o],
                                    pd.eint[o]);
    smax = s > smax ? s : smax;
  }
  smax = wave_max(smax);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) wmax[wid] = smax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = wmax[0];
    for (int i = 1; i < int(blockDim.x >> 6); ++i) m = wmax[i] > m ? wmax[i] : m;
    // non-negative doubles order like their bit patterns
    atomicMax(&smax_bits[pd.level], (unsigned long long)__double_as_longlong(m));
  }
}

// dt = kappa a / max signal (Eq. dthydro in comoving coordinates).
__global__ void cfl_finalize_kernel(int32_t nlevels, double cfl,
                                    const double *__restrict__ expand,
                                    unsigned long long *__restrict__ smax_bits,
                                    double *__restrict__ dt_dev) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nlevels) return;
  const double s = __longlong_as_double((long long)smax_bits[l]);
  const double ka = cfl * (expand ? expand[2 * l] : 1.0);
  dt_dev[l] = s > 0.0 ? ka / s : __longlong_as_double(0x7ff0000000000000LL);
  smax_bits[l] = 0ull;
}

// ---------------------------------------------------------------------------
// Expansion terms of the comoving equations (Sec. "Physical Equations"),
// split from the sweeps and integrated implicitly and time-centred over the
// level's dt with H = adot / a of the level: peculiar velocity times
// (1 - H dt/2)/(1 + H dt/2), specific total energy times (1 - H dt)/(1 + H dt),
// specific internal energy times (1 - x)/(1 + x) with x = 3 (gamma - 1) H dt / 2.
// Active cells only, chunked over the patches like the CFL reduction.
template <class Prec>
__global__ void __launch_bounds__(256)
expansion_kernel(const PatchDev *__restrict__ patches, const int32_t *__restrict__ chunk_start,
                 int32_t npatch, int32_t cells_per_block, double gamma,
                 const double *__restrict__ expand, const double *__restrict__ dt_dev) {
  using S = typename Prec::S;
  const int p = find_patch(chunk_start, npatch, blockIdx.x);
  const PatchDev pd = patches[p];
  const int g = pd.ghost;
  const int64_t nx = pd.n[0], ny = pd.n[1];
  const int64_t total = nx * ny * pd.n[2];
  const int64_t nfx = nx + 2 * g, nfy = ny + 2 * g;
  const int64_t c0 = int64_t(blockIdx.x - chunk_start[p]) * cells_per_block;
  const int64_t c1 = c0 + cells_per_block < total ? c0 + cells_per_block : total;
  const double a = expand[2 * pd.level], adot = expand[2 * pd.level + 1];
  const double dt = dt_dev[pd.level];
  const double H = adot / a;
  const double xv = 0.5 * H * dt, xE = H * dt, xe = 1.5 * (gamma - 1.0) * H * dt;
  const double fv = (1.0 - xv) / (1.0 + xv);
  const double fE = (1.0 - xE) / (1.0 + xE);
  const double fe = (1.0 - xe) / (1.0 + xe);
  S *vx = static_cast<S *>(pd.vel[0]);
  S *vy = static_cast<S *>(pd.vel[1]);
  S *vz = static_cast<S *>(pd.vel[2]);
  for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
    const int64_t x = c % nx, yz = c / nx;
    const int64_t y = yz % ny, z = yz / ny;
    const int64_t o = ((z + g) * nfy + (y + g)) * nfx + (x + g);
    vx[o] = S(double(vx[o]) * fv);
    vy[o] = S(double(vy[o]) * fv);
    vz[o] = S(double(vz[o]) * fv);
    pd.etot[o] = pd.etot[o] * fE;
    pd.eint[o] = pd.eint[o] * fe;
  }
}

// ---------------------------------------------------------------------------
// Ghost shell of a patch, cell t of shell_cells(): the two z slabs (full x,
// y), the two y slabs of the active z range (full x), then the two x slabs of
// the active y, z range.  False past the end.
__device__ __forceinline__ bool shell_cell(int g, const int64_t (&N)[3], const int64_t (&nf)[3],
                                           int64_t t, int64_t (&c)[3]) {
  const int64_t sz = 2 * g * nf[1] * nf[0];
  const int64_t sy = N[2] * 2 * g * nf[0];
  const int64_t sx = N[2] * N[1] * 2 * g;
  if (t >= sz + sy + sx) return false;
  if (t < sz) {
    c[0] = t % nf[0];
    c[1] = (t / nf[0]) % nf[1];
    const int64_t k = t / (nf[0] * nf[1]);
    c[2] = k < g ? k : N[2] + k;
  } else if (t < sz + sy) {
    const int64_t u = t - sz;
    c[0] = u % nf[0];
    const int64_t j = (u / nf[0]) % (2 * g);
    c[1] = j < g ? j : N[1] + j;
    c[2] = g + u / (nf[0] * 2 * g);
  } else {
    const int64_t u = t - sz - sy;
    const int64_t i = u % (2 * g);
    c[0] = i < g ? i : N[0] + i;
    c[1] = g + (u / (2 * g)) % N[1];
    c[2] = g + u / (2 * g * N[1]);
  }
  return true;
}

// ---------------------------------------------------------------------------
// Domain boundary fill of one patch (Sec. "Boundary conditions"): per face
// periodic, reflecting (mirror image, normal velocity reversed), outflow
// (copy of the edge cell) or inflow (fixed values).  The definition fills
// the axes in order x, y, z, each over the whole extent of the axes before it
// and the active range of the axes after it; a ghost cell is therefore
// written by its highest ghost axis from the cell that axis's rule points to,
// which is written the same way by its own highest ghost axis.  Each thread
// unrolls that chain for one shell cell: axes from z down to x, each ghost
// coordinate mapped by its face's rule (velocity flips collected on the
// way), an inflow face ending the chain with its values.
template <class Prec>
__global__ void __launch_bounds__(256)
fill_boundary_kernel(PatchDev pd, FaceRules fr) {
  using S = typename Prec::S;
  const int g = pd.ghost;
  const int64_t N[3] = {pd.n[0], pd.n[1], pd.n[2]};
  const int64_t nf[3] = {N[0] + 2 * g, N[1] + 2 * g, N[2] + 2 * g};
  int64_t c[3];
  if (!shell_cell(g, N, nf, int64_t(blockIdx.x) * blockDim.x + threadIdx.x, c)) return;
  int64_t sc[3] = {c[0], c[1], c[2]};
  bool flip[3] = {false, false, false};
  int inflow = -1;
  for (int a = 2; a >= 0; --a) {
    if (sc[a] >= g && sc[a] < g + N[a]) continue;
    const int side = sc[a] < g ? 0 : 1;
    const int kind = fr.kind[2 * a + side];
    if (kind == kFaceInflow) {
      inflow = 2 * a + side;
      break;
    }
    if (kind == kFacePeriodic) {
      sc[a] = g + (((sc[a] - g) % N[a]) + N[a]) % N[a];
    } else if (kind == kFaceReflecting) {
      sc[a] = side == 0 ? 2 * g - 1 - sc[a] : 2 * (g + N[a]) - 1 - sc[a];
      flip[a] = true;
    } else {
      sc[a] = side == 0 ? g : g + N[a] - 1;
    }
  }
  S *rho = static_cast<S *>(pd.rho);
  S *vel[3] = {static_cast<S *>(pd.vel[0]), static_cast<S *>(pd.vel[1]),
               static_cast<S *>(pd.vel[2])};
  const int64_t dst = (c[2] * nf[1] + c[1]) * nf[0] + c[0];
  S r, v[3];
  double E, e;
  if (inflow >= 0) {
    r = S(fr.inflow[inflow][0]);
    for (int a = 0; a < 3; ++a) v[a] = S(fr.inflow[inflow][1 + a]);
    E = fr.inflow[inflow][4];
    e = fr.inflow[inflow][5];
  } else {
    const int64_t src = (sc[2] * nf[1] + sc[1]) * nf[0] + sc[0];
    r = rho[src];
    for (int a = 0; a < 3; ++a) v[a] = vel[a][src];
    E = pd.etot[src];
    e = pd.eint[src];
  }
  rho[dst] = r;
  for (int a = 0; a < 3; ++a) vel[a][dst] = flip[a] ? -v[a] : v[a];
  pd.etot[dst] = E;
  pd.eint[dst] = e;
}

// ---------------------------------------------------------------------------
// Ghost cells of AMR patches from their parents and siblings (Sec. "Boundary
// conditions": interpolate every boundary cell from the parent, then copy
// from siblings wherever one covers it).
//
// SecondOrderA (Appendix "Interpolation", three-dimensional form) of one
// conserved quantity of the r^3 fine cells that refine the centre of
// nb[dz][dy][dx]: corner values are the averages of the 8 parent cells
// sharing a corner; slopes along the four diagonals are minmod-limited; if
// the change to corner (+,+,+) that dQ1..dQ3 imply leaves [0, dQ0] (s outside
// [0, 1]), the slopes pushing it out are scaled so that it lands on the near
// end (with dQ0 = 0: onto zero); the slopes are converted to the axes and
// evaluated at the fine cell centre.  Off the hot path, so divisions are the
// compiler's correctly rounded ones (exact also for subnormal operands).
__device__ __forceinline__ double minmod(double a, double b) {
  if (a * b < 0.0) return 0.0;
  const double m = fabs(a) < fabs(b) ? fabs(a) : fabs(b);
  return a < 0.0 ? -m : m;
}

// The eight 2x2x2 corner sums of a 3x3x3 neighbourhood, accumulated while
// its cells arrive in z, y, x order: corner (sx, sy, sz), index
// (sx > 0) + 2 (sy > 0) + 4 (sz > 0), holds the cells whose offsets lie on its
// side of the centre or at the centre along each axis, each sum starting
// from zero and taking its eight cells in that same z, y, x order.
struct CornerSums {
  double c[8];
  double centre;
};
__device__ __forceinline__ void corner_sums_begin(CornerSums &cs) {
#pragma unroll
  for (int n = 0; n < 8; ++n) cs.c[n] = 0.0;
}
template <int dz, int dy, int dx>
__device__ __forceinline__ void corner_sums_add(CornerSums &cs, double v) {
#pragma unroll
  for (int n = 0; n < 8; ++n) {
    const int sx = n & 1, sy = (n >> 1) & 1, sz = (n >> 2) & 1;  // 1: the + side
    const bool in_x = sx ? dx >= 1 : dx <= 1;
    const bool in_y = sy ? dy >= 1 : dy <= 1;
    const bool in_z = sz ? dz >= 1 : dz <= 1;
    if (in_x && in_y && in_z) cs.c[n] = cs.c[n] + v;
  }
  if (dz == 1 && dy == 1 && dx == 1) cs.centre = v;
}
__device__ __forceinline__ double corner_avg(const CornerSums &cs, int sx, int sy, int sz) {
  return cs.c[(sx > 0 ? 1 : 0) + (sy > 0 ? 2 : 0) + (sz > 0 ? 4 : 0)] * 0.125;
}

__device__ __forceinline__ void second_order_a_slopes(const CornerSums &cs, double &fx, double &fy,
                                                      double &fz) {
  const double q0 = cs.centre;
  const int c[4][3] = {{1, 1, 1}, {-1, 1, 1}, {1, -1, 1}, {1, 1, -1}};
  double dq[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    const double up = corner_avg(cs, c[n][0], c[n][1], c[n][2]);
    const double dn = corner_avg(cs, -c[n][0], -c[n][1], -c[n][2]);
    dq[n] = minmod(up - q0, q0 - dn);
  }
  const double sum = dq[1] + dq[2] + dq[3];
  bool adjust = false, chi[4] = {false, false, false, false};
  double target = 0.0;
  if (dq[0] != 0.0) {
    const double s = sum / dq[0];
    if (s < 0.0 || s > 1.0) {
      adjust = true;
      target = dq[0] * (s < 0.0 ? 0.0 : 1.0);
#pragma unroll
      for (int n = 1; n < 4; ++n) {
        const double ratio = dq[n] / dq[0];
        chi[n] = s < 0.0 ? ratio < 0.0 : ratio > 0.0;
      }
    }
  } else if (sum != 0.0) {
    adjust = true;
#pragma unroll
    for (int n = 1; n < 4; ++n) chi[n] = sum > 0.0 ? dq[n] > 0.0 : dq[n] < 0.0;
  }
  if (adjust) {
    double sel = 0.0, rest = 0.0;
#pragma unroll
    for (int n = 1; n < 4; ++n) {
      if (chi[n]) sel = sel + dq[n];
      else rest = rest + dq[n];
    }
    const double f = (target - rest) / sel;
#pragma unroll
    for (int n = 1; n < 4; ++n)
      if (chi[n]) dq[n] = f * dq[n];
  }
  fx = dq[2] + dq[3];
  fy = dq[1] + dq[3];
  fz = dq[1] + dq[2];
}

// The interpolant at fine cell (i, j, k) of the r^3 that refine the centre.
__device__ __forceinline__ double second_order_a_eval(double q0, double fx, double fy, double fz,
                                                      int r, int i, int j, int k) {
  const double wx = (double(i) + (1.0 - r) * 0.5) / double(r);
  const double wy = (double(j) + (1.0 - r) * 0.5) / double(r);
  const double wz = (double(k) + (1.0 - r) * 0.5) / double(r);
  return q0 + wx * fx + wy * fy + wz * fz;
}

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
  return a >= 0 ? a / b : -((-a + b - 1) / b);
}

__device__ __forceinline__ int find_item(const int64_t *prefix, int32_t n, int64_t t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One thread per parent cell that a listed box's cells refine (the box of
// such cells in the parent's level, in x-fastest order): the 27-cell
// neighbourhood of rho, rho v, rho E, rho e around it (the density read once,
// each quantity folded into its eight corner sums as its cells are read, so
// no quantity's neighbourhood is held whole), the SecondOrderA slopes of
// each, and for every one of its r^3 fine cells inside the box the
// interpolant's values, stored as rho, v = (rho v)/rho, E, e.  A parent cell
// whose fine cells fall in two boxes is interpolated by both, to the same
// values.  The parent's state is read through parent_tab[parent] when given
// (the parent blended in time), else from the patch table.
template <class Prec>
__global__ void __launch_bounds__(256, 2)
fill_from_parent_kernel(const PatchDev *__restrict__ patches, const InterpItem *__restrict__ items,
                        const int64_t *__restrict__ prefix, int32_t nitems, int64_t total,
                        const PatchDev *__restrict__ parent_tab) {
  using S = typename Prec::S;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int it = find_item(prefix, nitems, t);
  const InterpItem item = items[it];
  const PatchDev fd = patches[item.patch];
  const PatchDev cd = parent_tab ? parent_tab[item.parent] : patches[item.parent];
  const int gf = fd.ghost, gc = cd.ghost, r = item.r;
  const int64_t nf[3] = {int64_t(fd.n[0]) + 2 * gf, int64_t(fd.n[1]) + 2 * gf,
                         int64_t(fd.n[2]) + 2 * gf};
  const int64_t nc[3] = {int64_t(cd.n[0]) + 2 * gc, int64_t(cd.n[1]) + 2 * gc,
                         int64_t(cd.n[2]) + 2 * gc};
  int64_t clo[3], cext[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    clo[a] = floor_div(int64_t(item.start[a]) + item.lo[a] - gf, r);
    cext[a] = floor_div(int64_t(item.start[a]) + item.hi[a] - 1 - gf, r) - clo[a] + 1;
  }
  const int64_t u = t - prefix[it];
  const int64_t cc[3] = {clo[0] + u % cext[0], clo[1] + (u / cext[0]) % cext[1],
                         clo[2] + u / (cext[0] * cext[1])};
  // local index of the first of its fine cells in the patch; which are in the box
  int64_t f0[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) f0[a] = cc[a] * r - item.start[a] + gf;
  auto in_box = [&](int i, int j, int k) {
    const int64_t f[3] = {f0[0] + i, f0[1] + j, f0[2] + k};
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) in = in && f[a] >= item.lo[a] && f[a] < item.hi[a];
    return in;
  };
  int64_t lc[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) lc[a] = cc[a] - item.pstart[a] + gc;
  const int64_t o0 = ((lc[2] - 1) * nc[1] + (lc[1] - 1)) * nc[0] + (lc[0] - 1);
  const S *rho_c = static_cast<const S *>(cd.rho);
  // the density of the neighbourhood, read once for all six quantities
  double rn[27];
  auto cell = [&](int dz, int dy, int dx) __attribute__((always_inline)) {
    return o0 + (dz * nc[1] + dy) * nc[0] + dx;
  };
#pragma unroll
  for (int m = 0; m < 27; ++m) rn[m] = double(rho_c[cell(m / 9, (m / 3) % 3, m % 3)]);
  // one quantity's slopes from its neighbourhood: rho (comp 0), then rho times
  // the stored field (velocities, E, e), folded into the corner sums as read
  auto slopes = [&](int comp, double &q0, double &fx, double &fy,
                    double &fz) __attribute__((always_inline)) {
    // (pointers picked by value, not by a run-time index into the table's
    // arrays, which would put the table in scratch memory)
    const S *xs = comp == 1   ? static_cast<const S *>(cd.vel[0])
                  : comp == 2 ? static_cast<const S *>(cd.vel[1])
                  : comp == 3 ? static_cast<const S *>(cd.vel[2])
                              : nullptr;
    const double *xd = comp == 4 ? cd.etot : cd.eint;
    CornerSums cs;
    corner_sums_begin(cs);
    auto value = [&](int m) __attribute__((always_inline)) {
      if (comp == 0) return rn[m];
      const int64_t o = cell(m / 9, (m / 3) % 3, m % 3);
      return rn[m] * (xs ? double(xs[o]) : xd[o]);
    };
#define PPM_CORNER_CELL(DZ, DY, DX) corner_sums_add<DZ, DY, DX>(cs, value(DZ * 9 + DY * 3 + DX))
#define PPM_CORNER_ROW(DZ, DY) \
  PPM_CORNER_CELL(DZ, DY, 0); PPM_CORNER_CELL(DZ, DY, 1); PPM_CORNER_CELL(DZ, DY, 2)
#define PPM_CORNER_PLANE(DZ) PPM_CORNER_ROW(DZ, 0); PPM_CORNER_ROW(DZ, 1); PPM_CORNER_ROW(DZ, 2)
    PPM_CORNER_PLANE(0);
    PPM_CORNER_PLANE(1);
    PPM_CORNER_PLANE(2);
#undef PPM_CORNER_PLANE
#undef PPM_CORNER_ROW
#undef PPM_CORNER_CELL
    q0 = cs.centre;
    second_order_a_slopes(cs, fx, fy, fz);
  };
  double q0[6], fx[6], fy[6], fz[6];
#pragma unroll
  for (int comp = 0; comp < 6; ++comp) slopes(comp, q0[comp], fx[comp], fy[comp], fz[comp]);
  S *rho_p = static_cast<S *>(fd.rho);
  S *vel[3] = {static_cast<S *>(fd.vel[0]), static_cast<S *>(fd.vel[1]),
               static_cast<S *>(fd.vel[2])};
  for (int k = 0; k < r; ++k)
    for (int j = 0; j < r; ++j)
      for (int i = 0; i < r; ++i) {
        if (!in_box(i, j, k)) continue;
        double q[6];
#pragma unroll
        for (int comp = 0; comp < 6; ++comp)
          q[comp] = second_order_a_eval(q0[comp], fx[comp], fy[comp], fz[comp], r, i, j, k);
        const int64_t dst = ((f0[2] + k) * nf[1] + (f0[1] + j)) * nf[0] + (f0[0] + i);
        rho_p[dst] = S(q[0]);
#pragma unroll
        for (int a = 0; a < 3; ++a) vel[a][dst] = S(q[1 + a] / q[0]);
        fd.etot[dst] = q[4] / q[0];
        fd.eint[dst] = q[5] / q[0];
      }
}

// One thread per cell of the listed boxes: the sibling's value, unless the
// cell is active in its own patch.
template <class Prec>
__global__ void __launch_bounds__(256)
copy_from_siblings_kernel(const PatchDev *__restrict__ patches, const SiblingBox *__restrict__ boxes,
                          const int64_t *__restrict__ prefix, int32_t nboxes, int64_t total) {
  using S = typename Prec::S;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int b = find_item(prefix, nboxes, t);
  const SiblingBox box = boxes[b];
  const int64_t u = t - prefix[b];
  const int64_t ex = box.hi[0] - box.lo[0], ey = box.hi[1] - box.lo[1];
  const int64_t c[3] = {box.lo[0] + u % ex, box.lo[1] + (u / ex) % ey, box.lo[2] + u / (ex * ey)};
  const PatchDev dd = patches[box.dst];
  const PatchDev sd = patches[box.src];
  const int gd = dd.ghost, gs = sd.ghost;
  bool active = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) active = active && c[a] >= gd && c[a] < gd + dd.n[a];
  if (active) return;
  const int64_t nd[3] = {int64_t(dd.n[0]) + 2 * gd, int64_t(dd.n[1]) + 2 * gd,
                         int64_t(dd.n[2]) + 2 * gd};
  const int64_t ns[3] = {int64_t(sd.n[0]) + 2 * gs, int64_t(sd.n[1]) + 2 * gs,
                         int64_t(sd.n[2]) + 2 * gs};
  const int64_t sc[3] = {c[0] + box.shift[0], c[1] + box.shift[1], c[2] + box.shift[2]};
  const int64_t dst = (c[2] * nd[1] + c[1]) * nd[0] + c[0];
  const int64_t src = (sc[2] * ns[1] + sc[1]) * ns[0] + sc[0];
  static_cast<S *>(dd.rho)[dst] = static_cast<const S *>(sd.rho)[src];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    static_cast<S *>(dd.vel[a])[dst] = static_cast<const S *>(sd.vel[a])[src];
  dd.etot[dst] = sd.etot[src];
  dd.eint[dst] = sd.eint[src];
}

// ---------------------------------------------------------------------------
// AMR level step: the coarse fluxes through the faces of child footprints,
// the fine registers summed over substeps, flux correction and projection
// (Secs. "Flux correction" and "Projection").

// Captured faces, six per wavefront: lanes 10w .. 10w+9 hold cells j-4 ..
// j+5 of row w's pencil (j the cell left of the face) and run the
// lane-parallel segment code, which yields the same final flux for the face
// as the sweep that follows.  The flux through face j+1/2, fallback
// included, depends only on those ten cells: the Riemann states of faces
// j-1/2 .. j+3/2 use cells j-4 .. j+5 (the flattening of a cell looks two
// cells out, and the neighbour whose flattening it may take one more), and
// the fallback tests the provisional updates of cells j and j+1.  So what a
// window's edge lanes read from the adjacent window never reaches that face.
// Nothing is written but dt F of the face.
constexpr int kCapWindow = 10, kCapPerWave = 6;

template <class Prec, bool kUseHLLC, bool kGrav>
__global__ void __launch_bounds__(256)
capture_kernel(const PatchDev *__restrict__ patches, const CaptureRow *__restrict__ rows,
               int32_t nrows, int32_t axis, const double *__restrict__ dt_dev, Params P) {
  using S = typename Prec::S;
  const int row0 = (int(blockIdx.x) * 4 + int(threadIdx.x >> 6)) * kCapPerWave;
  if (row0 >= nrows) return;  // the whole wave leaves
  const int lane = threadIdx.x & 63;
  const int slot = lane / kCapWindow, pos = lane - slot * kCapWindow;
  const bool used = slot < kCapPerWave && row0 + slot < nrows;
  const CaptureRow cr = rows[used ? row0 + slot : row0];
  const PatchDev pd = patches[cr.patch];
  PencilRef<S> pc = make_pencil<S>(pd, axis, cr.i1, cr.i2);
  pc.reg_lo = pc.reg_hi = nullptr;
  const double dt = dt_dev[pd.level];
  const double a = expansion_a(P, pd.level);
  const double lam = dt / (a * pc.dx);
  const double hgdt = 0.5 * dt / a;
  const int jc = cr.j - 4 + pos;
  const bool in = used && jc >= 0 && jc < pc.n;
  const int j = in ? jc : -1;
  CellLoad cur = {1.0, 0.0, 0.0, 0.0, 1.0, 1.0};
  if (in) {
    const int64_t o = pc.base + int64_t(j) * pc.stride;
    cur.r = double(pc.rho[o]); cur.u = double(pc.u[o]);
    cur.v1 = double(pc.v1[o]); cur.v2 = double(pc.v2[o]);
    cur.E = pc.E[o]; cur.e = pc.e[o];
  }
  uint32_t nfb = 0, nfl = 0;
  CflAcc cfl = cfl_acc(pd, axis, nullptr);
  // the face's final flux reads the provisional fluxes of faces j-1/2 ..
  // j+3/2 (the fallback tests of cells j and j+1)
  const bool need_face = pos >= 3 && pos <= 5;
  const auto F = sweep_segment<Prec, false, kUseHLLC, kGrav>(P, pc, dt, lam, hgdt, j, false,
                                                             need_face, cur, nfb, nfl, cfl);
  if (used && pos == 4) {
#pragma unroll
    for (int k = 0; k < 6; ++k) cr.dst[pc.lab[k] * cr.fstride] = dt * F.get(k);
  }
}

// One thread per cell of the listed boxes, all six fields (see
// launch_box_state).
template <class Prec, bool kBlend>
__global__ void __launch_bounds__(256)
box_state_kernel(const PatchDev *__restrict__ cur_tab, const PatchDev *__restrict__ old_tab,
                 const PatchDev *__restrict__ mid_tab, const CellBox *__restrict__ boxes,
                 const int64_t *__restrict__ prefix, int32_t nboxes, int64_t total, double w) {
  using S = typename Prec::S;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int b = find_item(prefix, nboxes, t);
  const CellBox box = boxes[b];
  const int64_t u = t - prefix[b];
  const int64_t ex = box.hi[0] - box.lo[0], ey = box.hi[1] - box.lo[1];
  const int64_t c[3] = {box.lo[0] + u % ex, box.lo[1] + (u / ex) % ey, box.lo[2] + u / (ex * ey)};
  const PatchDev cd = cur_tab[box.patch];
  const PatchDev od = old_tab[box.patch];
  const int64_t g = cd.ghost;
  const int64_t nx = cd.n[0] + 2 * g, ny = cd.n[1] + 2 * g;
  const int64_t o = (c[2] * ny + c[1]) * nx + c[0];
  const S *cs[4] = {static_cast<const S *>(cd.rho), static_cast<const S *>(cd.vel[0]),
                    static_cast<const S *>(cd.vel[1]), static_cast<const S *>(cd.vel[2])};
  S *os[4] = {static_cast<S *>(od.rho), static_cast<S *>(od.vel[0]),
              static_cast<S *>(od.vel[1]), static_cast<S *>(od.vel[2])};
  if (!kBlend) {
#pragma unroll
    for (int f = 0; f < 4; ++f) os[f][o] = cs[f][o];
    od.etot[o] = cd.etot[o];
    od.eint[o] = cd.eint[o];
    return;
  }
  const PatchDev md = mid_tab[box.patch];
  S *ms[4] = {static_cast<S *>(md.rho), static_cast<S *>(md.vel[0]),
              static_cast<S *>(md.vel[1]), static_cast<S *>(md.vel[2])};
  const double wo = 1.0 - w;
#pragma unroll
  for (int f = 0; f < 4; ++f) ms[f][o] = S(wo * double(os[f][o]) + w * double(cs[f][o]));
  md.etot[o] = wo * od.etot[o] + w * cd.etot[o];
  md.eint[o] = wo * od.eint[o] + w * cd.eint[o];
}

__global__ void __launch_bounds__(256)
accumulate_kernel(const AccItem *__restrict__ items, const int64_t *__restrict__ prefix,
                  int32_t nitems, int64_t total) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int it = find_item(prefix, nitems, t);
  const AccItem item = items[it];
  const int64_t u = t - prefix[it];
  item.acc[u] = item.acc[u] + item.reg[u];
}

// One thread per corrected coarse cell: the changes of rho, rho v, rho E,
// rho e from each face it shares with a child footprint (coarse flux minus
// the area average of the fine fluxes, over a dx, signed by the side),
// summed in list order, then applied to the conserved quantities and stored.
template <class Prec>
__global__ void __launch_bounds__(256)
flux_correct_kernel(const PatchDev *__restrict__ patches, const CorrTarget *__restrict__ targets,
                    int32_t ntargets, const CorrContrib *__restrict__ contribs, Params P) {
  using S = typename Prec::S;
  const int t = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= ntargets) return;
  const CorrTarget tg = targets[t];
  const PatchDev pd = patches[tg.patch];
  const double a = expansion_a(P, pd.level);
  double dq[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int c = tg.first; c < tg.first + tg.count; ++c) {
    const CorrContrib cb = contribs[c];
    const double rr = double(cb.r * cb.r);
    for (int k = 0; k < 6; ++k) {
      double sum = 0.0;
      for (int jj = 0; jj < cb.r; ++jj)
        for (int ii = 0; ii < cb.r; ++ii)
          sum += cb.fine[k * cb.fine_fstride + int64_t(jj) * cb.fine_row + ii];
      const double fine = sum / rr;
      const double coarse = cb.cap[k * cb.cap_fstride];
      const double d = cb.side == 0 ? coarse - fine : fine - coarse;
      dq[k] += d / (a * pd.dx[cb.axis]);
    }
  }
  const int64_t o = tg.cell;
  S *rho_p = static_cast<S *>(pd.rho);
  S *vx = static_cast<S *>(pd.vel[0]);
  S *vy = static_cast<S *>(pd.vel[1]);
  S *vz = static_cast<S *>(pd.vel[2]);
  const double rho = double(rho_p[o]);
  const double rn = rho + dq[0];
  const double mx = rho * double(vx[o]) + dq[1];
  const double my = rho * double(vy[o]) + dq[2];
  const double mz = rho * double(vz[o]) + dq[3];
  const double mE = rho * pd.etot[o] + dq[4];
  const double me = rho * pd.eint[o] + dq[5];
  rho_p[o] = S(rn);
  vx[o] = S(mx / rn);
  vy[o] = S(my / rn);
  vz[o] = S(mz / rn);
  pd.etot[o] = mE / rn;
  pd.eint[o] = me / rn;
}

// One thread per coarse cell of a child footprint: the volume average of the
// conserved quantities of the r^3 fine cells over it.
template <class Prec>
__global__ void __launch_bounds__(256)
project_kernel(const PatchDev *__restrict__ patches, const ProjItem *__restrict__ items,
               const int64_t *__restrict__ prefix, int32_t nitems, int64_t total) {
  using S = typename Prec::S;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int it = find_item(prefix, nitems, t);
  const ProjItem item = items[it];
  const int64_t u = t - prefix[it];
  const int64_t ex = item.hi[0] - item.lo[0], ey = item.hi[1] - item.lo[1];
  const int64_t x = item.lo[0] + u % ex, y = item.lo[1] + (u / ex) % ey;
  const int64_t z = item.lo[2] + u / (ex * ey);
  const PatchDev cd = patches[item.coarse];
  const PatchDev fd = patches[item.fine];
  const int gc = cd.ghost, gf = fd.ghost, r = item.r;
  const int64_t nc[2] = {int64_t(cd.n[0]) + 2 * gc, int64_t(cd.n[1]) + 2 * gc};
  const int64_t nf[2] = {int64_t(fd.n[0]) + 2 * gf, int64_t(fd.n[1]) + 2 * gf};
  const S *frho = static_cast<const S *>(fd.rho);
  const S *fv[3] = {static_cast<const S *>(fd.vel[0]), static_cast<const S *>(fd.vel[1]),
                    static_cast<const S *>(fd.vel[2])};
  double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int kk = 0; kk < r; ++kk)
    for (int jj = 0; jj < r; ++jj)
      for (int ii = 0; ii < r; ++ii) {
        const int64_t fx = gf + (x - item.lo[0]) * r + ii;
        const int64_t fy = gf + (y - item.lo[1]) * r + jj;
        const int64_t fz = gf + (z - item.lo[2]) * r + kk;
        const int64_t o = (fz * nf[1] + fy) * nf[0] + fx;
        const double rho = double(frho[o]);
        s[0] += rho;
        s[1] += rho * double(fv[0][o]);
        s[2] += rho * double(fv[1][o]);
        s[3] += rho * double(fv[2][o]);
        s[4] += rho * fd.etot[o];
        s[5] += rho * fd.eint[o];
      }
  const double vol = double(r * r * r);
  const int64_t o = ((z + gc) * nc[1] + (y + gc)) * nc[0] + (x + gc);
  const double rho = s[0] / vol;
  static_cast<S *>(cd.rho)[o] = S(rho);
  static_cast<S *>(cd.vel[0])[o] = S((s[1] / vol) / rho);
  static_cast<S *>(cd.vel[1])[o] = S((s[2] / vol) / rho);
  static_cast<S *>(cd.vel[2])[o] = S((s[3] / vol) / rho);
  cd.etot[o] = (s[4] / vol) / rho;
  cd.eint[o] = (s[5] / vol) / rho;
}

// ---------------------------------------------------------------------------
// Periodic ghost fill of one patch: only ghost cells are visited.  The shell
// is split into the two z slabs (full x, y), the two y slabs of the active z
// range (full x), and the two x slabs of the active y, z range.

template <class Prec>
__global__ void __launch_bounds__(256)
fill_periodic_kernel(PatchDev pd) {
  using S = typename Prec::S;
  const int g = pd.ghost;
  const int64_t N[3] = {pd.n[0], pd.n[1], pd.n[2]};
  const int64_t nf[3] = {N[0] + 2 * g, N[1] + 2 * g, N[2] + 2 * g};
  int64_t c[3];
  if (!shell_cell(g, N, nf, int64_t(blockIdx.x) * blockDim.x + threadIdx.x, c)) return;
  const int64_t x = c[0], y = c[1], z = c[2];
  auto wrap = [&](int64_t i, int d) { return g + (((i - g) % N[d]) + N[d]) % N[d]; };
  const int64_t dst = (z * nf[1] + y) * nf[0] + x;
  const int64_t src = (wrap(z, 2) * nf[1] + wrap(y, 1)) * nf[0] + wrap(x, 0);
  S *rho = static_cast<S *>(pd.rho);
  S *vx = static_cast<S *>(pd.vel[0]);
  S *vy = static_cast<S *>(pd.vel[1]);
  S *vz = static_cast<S *>(pd.vel[2]);
  rho[dst] = rho[src];
  vx[dst] = vx[src];
  vy[dst] = vy[src];
  vz[dst] = vz[src];
  pd.etot[dst] = pd.etot[src];
  pd.eint[dst] = pd.eint[src];
}

// ---------------------------------------------------------------------------
// Launchers

#endif  // PPM_PASS_FP64

// The three builds of each sweep kernel (template arguments kUseHLLC, kGrav):
// two-shock only; HLLC or two-shock as the flag says; the general build,
// which adds the gravity source terms and the diffusive flux, for plans where
// some patch has an acceleration field or the diffusive flux is on.
#define PPM_BUILD(P, LAUNCH, ...)                                              \
  if ((P).flags & (kAnyGravity | kDiffusion)) LAUNCH(__VA_ARGS__, true, true); \
  else if ((P).flags & kHLLC) LAUNCH(__VA_ARGS__, true, false);                \
  else LAUNCH(__VA_ARGS__, false, false)

template <class Prec>
hipError_t launch_sweep(const PatchDev *patches, const int32_t *chunk_start, int32_t npatch,
                        int32_t nblocks, int32_t block, int32_t axis, int32_t mask,
                        const double *dt_dev, const Params &P, unsigned long long *counters,
                        unsigned long long *smax_bits, const int32_t *groups, int32_t ngroups,
                        hipStream_t s, double *defer) {
  const size_t lds = size_t(kLdsMarch + (smax_bits ? 1 : 0)) * block * sizeof(double);
#define PPM_LAUNCH_MARCH(CFL, GRP, HLLC, GRAV)                                               \
  hipLaunchKernelGGL((sweep_kernel<Prec, CFL, GRP, HLLC, GRAV>), dim3(nblocks), dim3(block), \
                     lds, s, patches, chunk_start, npatch, axis, mask, dt_dev, P, counters,   \
                     smax_bits, groups, ngroups)
#define PPM_LAUNCH_SPLIT(CFL, HLLC, GRAV)                                                      \
  hipLaunchKernelGGL((sweep_split_kernel<Prec, CFL, HLLC, GRAV>), dim3(nblocks), dim3(block),  \
                     lds, s, patches, axis, mask, dt_dev, P, counters, smax_bits, defer)
  if (defer) {
    if (smax_bits) { PPM_BUILD(P, PPM_LAUNCH_SPLIT, true); }
    else { PPM_BUILD(P, PPM_LAUNCH_SPLIT, false); }
  } else if (groups) {
    if (smax_bits) { PPM_BUILD(P, PPM_LAUNCH_MARCH, true, true); }
    else { PPM_BUILD(P, PPM_LAUNCH_MARCH, false, true); }
  } else {
    if (smax_bits) { PPM_BUILD(P, PPM_LAUNCH_MARCH, true, false); }
    else { PPM_BUILD(P, PPM_LAUNCH_MARCH, false, false); }
  }
#undef PPM_LAUNCH_MARCH
#undef PPM_LAUNCH_SPLIT
  return hipGetLastError();
}

template <class Prec>
hipError_t launch_sweep_lanes(const PatchDev *patches, const int32_t *chunk_start, int32_t npatch,
                              int32_t nblocks, int32_t block, int32_t axis, int32_t mask,
                              const double *dt_dev, const Params &P,
                              unsigned long long *counters, unsigned long long *smax_bits,
                              hipStream_t s) {
#define PPM_LAUNCH_LANES(CFL, HLLC, GRAV)                                                    \
  hipLaunchKernelGGL((sweep_lanes_kernel<Prec, CFL, HLLC, GRAV>), dim3(nblocks), dim3(block), \
                     0, s, patches, chunk_start, npatch, axis, mask, dt_dev, P, counters,      \
                     smax_bits)
  if (smax_bits) { PPM_BUILD(P, PPM_LAUNCH_LANES, true); }
  else { PPM_BUILD(P, PPM_LAUNCH_LANES, false); }
#undef PPM_LAUNCH_LANES
  return hipGetLastError();
}

template <class Prec>
hipError_t launch_sweep_tail(const PatchDev *patches, const int32_t *chunk_start, int32_t nblocks,
                             int32_t block, int32_t axis, int32_t mask, int32_t pencil0,
                             const double *dt_dev, const Params &P, unsigned long long *counters,
                             unsigned long long *smax_bits, hipStream_t s) {
#define PPM_LAUNCH_TAIL(CFL, HLLC, GRAV)                                                     \
  hipLaunchKernelGGL((sweep_tail_kernel<Prec, CFL, HLLC, GRAV>), dim3(nblocks), dim3(block),  \
                     0, s, patches, chunk_start, axis, mask, pencil0, dt_dev, P, counters,     \
                     smax_bits)
  if (smax_bits) { PPM_BUILD(P, PPM_LAUNCH_TAIL, true); }
  else { PPM_BUILD(P, PPM_LAUNCH_TAIL, false); }
#undef PPM_LAUNCH_TAIL
  return hipGetLastError();
}

template <class Prec>
hipError_t launch_batch(const PatchDev *patches, const int32_t *order, int32_t npatch,
                        int32_t nblocks, int32_t block, int32_t sweep_order, int32_t lanes_mask,
                        const double *dt_dev, const Params &P, unsigned long long *counters,
                        unsigned int *queue, unsigned long long *smax_bits, hipStream_t s) {
  const size_t lds = size_t(kLdsMarch + (smax_bits ? 1 : 0)) * block * sizeof(double);
#define PPM_LAUNCH_BATCH(CFL, HLLC, GRAV)                                                    \
  hipLaunchKernelGGL((batch_persistent_kernel<Prec, CFL, HLLC, GRAV>), dim3(nblocks),         \
                     dim3(block), lds, s, patches, order, npatch, sweep_order, lanes_mask,     \
                     dt_dev, P, counters, queue, smax_bits)
  if (smax_bits) { PPM_BUILD(P, PPM_LAUNCH_BATCH, true); }
  else { PPM_BUILD(P, PPM_LAUNCH_BATCH, false); }
#undef PPM_LAUNCH_BATCH
  return hipGetLastError();
}
#undef PPM_BUILD

#if PPM_PASS_FP64
template <class Prec>
hipError_t launch_expansion(const PatchDev *patches, const int32_t *chunk_start, int32_t npatch,
                            int32_t nblocks, int32_t cells_per_block, double gamma,
                            const double *expand, const double *dt_dev, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(expansion_kernel<Prec>, dim3(nblocks), dim3(256), 0, s, patches,
                     chunk_start, npatch, cells_per_block, gamma, expand, dt_dev);
  return hipGetLastError();
}

hipError_t launch_cfl_finalize(int32_t nlevels, double cfl, const double *expand,
                               unsigned long long *smax_bits, double *dt_dev, hipStream_t s) {
  hipLaunchKernelGGL(cfl_finalize_kernel, dim3((nlevels + 63) / 64), dim3(64), 0, s, nlevels,
                     cfl, expand, smax_bits, dt_dev);
  return hipGetLastError();
}

template <class Prec>
hipError_t launch_cfl(const PatchDev *patches, const int32_t *chunk_start, int32_t npatch,
                      int32_t nblocks, int32_t cells_per_block, int32_t nlevels, const Params &P,
                      unsigned long long *smax_bits, double *dt_dev, hipStream_t s) {
  hipLaunchKernelGGL(cfl_reduce_kernel<Prec>, dim3(nblocks), dim3(256), 0, s, patches,
                     chunk_start, npatch, cells_per_block, P, smax_bits);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_cfl_finalize(nlevels, P.cfl, P.expand, smax_bits, dt_dev, s);
}

template <class Prec>
hipError_t launch_fill_boundary(const PatchDev &pd, const FaceRules &fr, hipStream_t s) {
  const int64_t g = pd.ghost;
  const int64_t N[3] = {pd.n[0], pd.n[1], pd.n[2]};
  const int64_t nf[3] = {N[0] + 2 * g, N[1] + 2 * g, N[2] + 2 * g};
  const int64_t total = 2 * g * nf[1] * nf[0] + N[2] * 2 * g * nf[0] + N[2] * N[1] * 2 * g;
  const int64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL(fill_boundary_kernel<Prec>, dim3(unsigned(blocks)), dim3(256), 0, s, pd, fr);
  return hipGetLastError();
}

template <class Prec>
hipError_t launch_fill_from_parent(const PatchDev *patches, const InterpItem *items,
                                   const int64_t *prefix, int32_t nitems, int64_t total,
                                   const PatchDev *parent_tab, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_from_parent_kernel<Prec>, dim3(unsigned((total + 255) / 256)),
                     dim3(256), 0, s, patches, items, prefix, nitems, total, parent_tab);
  return hipGetLastError();
}

template <class Prec>
hipError_t launch_capture(const PatchDev *patches, const CaptureRow *rows, int32_t nrows,
                          int32_t axis, const double *dt_dev, const Params &P, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  const int64_t waves = (int64_t(nrows) + kCapPerWave - 1) / kCapPerWave;
  const unsigned blocks = unsigned((waves + 3) / 4);
#define PPM_LAUNCH_CAPTURE(HLLC, GRAV)                                                       \
  hipLaunchKernelGGL((capture_kernel<Prec, HLLC, GRAV>), dim3(blocks), dim3(256), 0, s,       \
                     patches, rows, nrows, axis, dt_dev, P)
  if (P.flags & (kAnyGravity | kDiffusion)) PPM_LAUNCH_CAPTURE(true, true);
  else if (P.flags & kHLLC) PPM_LAUNCH_CAPTURE(true, false);
  else PPM_LAUNCH_CAPTURE(false, false);
#undef PPM_LAUNCH_CAPTURE
  return hipGetLastError();
}

template <class Prec>
hipError_t launch_box_state(const PatchDev *cur, const PatchDev *old, const PatchDev *mid,
                            const CellBox *boxes, const int64_t *prefix, int32_t nboxes,
                            int64_t total, bool blend, double w, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  const dim3 grid(unsigned((total + 255) / 256));
  if (blend)
    hipLaunchKernelGGL((box_state_kernel<Prec, true>), grid, dim3(256), 0, s, cur, old, mid,
                       boxes, prefix, nboxes, total, w);
  else
    hipLaunchKernelGGL((box_state_kernel<Prec, false>), grid, dim3(256), 0, s, cur, old, mid,
                       boxes, prefix, nboxes, total, w);
  return hipGetLastError();
}

hipError_t launch_accumulate(const AccItem *items, const int64_t *prefix, int32_t nitems,
                             int64_t total, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(accumulate_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s,
                     items, prefix, nitems, total);
  return hipGetLastError();
}

template <class Prec>
hipError_t launch_flux_correct(const PatchDev *patches, const CorrTarget *targets,
                               int32_t ntargets, const CorrContrib *contribs, const Params &P,
                               hipStream_t s) {
  if (ntargets <= 0) return hipSuccess;
  hipLaunchKernelGGL(flux_correct_kernel<Prec>, dim3(unsigned((ntargets + 255) / 256)), dim3(256),
                     0, s, patches, targets, ntargets, contribs, P);
  return hipGetLastError();
}

template <class Prec>
hipError_t launch_project(const PatchDev *patches, const ProjItem *items, const int64_t *prefix,
                          int32_t nitems, int64_t total, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(project_kernel<Prec>, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s,
                     patches, items, prefix, nitems, total);
  return hipGetLastError();
}

template <class Prec>
hipError_t launch_copy_from_siblings(const PatchDev *patches, const SiblingBox *boxes,
                                     const int64_t *prefix, int32_t nboxes, int64_t total,
                                     hipStream_t s) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_from_siblings_kernel<Prec>, dim3(unsigned((total + 255) / 256)),
                     dim3(256), 0, s, patches, boxes, prefix, nboxes, total);
  return hipGetLastError();
}

template <class Prec>
hipError_t launch_fill(const PatchDev &pd, hipStream_t s) {
  const int64_t g = pd.ghost;
  const int64_t N[3] = {pd.n[0], pd.n[1], pd.n[2]};
  const int64_t nf[3] = {N[0] + 2 * g, N[1] + 2 * g, N[2] + 2 * g};
  const int64_t total = 2 * g * nf[1] * nf[0] + N[2] * 2 * g * nf[0] + N[2] * N[1] * 2 * g;
  const int64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL(fill_periodic_kernel<Prec>, dim3(unsigned(blocks)), dim3(256), 0, s, pd);
  return hipGetLastError();
}
#endif  // PPM_PASS_FP64

#define PPM_INSTANTIATE_MARCH(Prec)                                                            \
  template hipError_t launch_sweep<Prec>(const PatchDev *, const int32_t *, int32_t, int32_t,     \
                                         int32_t, int32_t, int32_t, const double *,               \
                                         const Params &, unsigned long long *,                    \
                                         unsigned long long *, const int32_t *, int32_t,          \
                                         hipStream_t, double *);                                   \
  template hipError_t launch_batch<Prec>(const PatchDev *, const int32_t *, int32_t, int32_t,     \
                                         int32_t, int32_t, int32_t, const double *,               \
                                         const Params &, unsigned long long *, unsigned int *,    \
                                         unsigned long long *, hipStream_t);
#define PPM_INSTANTIATE_LANES(Prec)                                                            \
  template hipError_t launch_sweep_lanes<Prec>(const PatchDev *, const int32_t *, int32_t,        \
                                               int32_t, int32_t, int32_t, int32_t,                \
                                               const double *, const Params &,                    \
                                               unsigned long long *, unsigned long long *,        \
                                               hipStream_t);                                       \
  template hipError_t launch_sweep_tail<Prec>(const PatchDev *, const int32_t *, int32_t, int32_t, \
                                              int32_t, int32_t, int32_t, const double *,          \
                                              const Params &, unsigned long long *,               \
                                              unsigned long long *, hipStream_t);
#if PPM_PASS_FP64
PPM_INSTANTIATE_MARCH(PrecF64)
#endif
#if PPM_PASS_FP64_LANES
PPM_INSTANTIATE_LANES(PrecF64)
#endif
#if PPM_PASS_MIXED
PPM_INSTANTIATE_MARCH(PrecMixed)
#endif
#if PPM_PASS_MIXED_LANES
PPM_INSTANTIATE_LANES(PrecMixed)
#endif
#undef PPM_INSTANTIATE_MARCH
#undef PPM_INSTANTIATE_LANES
#if PPM_PASS_FP64
__global__ void __launch_bounds__(256)
fp64_ops_kernel(const double *a, const double *b, double *quot, double *root, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  quot[i] = ddiv(a[i], b[i]);
  root[i] = dsqrt(a[i]);
}

hipError_t launch_fp64_ops(const double *a, const double *b, double *quot, double *root,
                           int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(fp64_ops_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, a, b, quot, root,
                     n);
  return hipGetLastError();
}

// Up to kWordBlock 32-bit words by value.
constexpr int kWordBlock = 240;
struct WordBlock {
  uint32_t w[kWordBlock];
};

__global__ void __launch_bounds__(256)
write_words_kernel(uint32_t *__restrict__ dst, WordBlock blk, int32_t n) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = blk.w[i];
}

hipError_t launch_write_words(uint32_t *dst, const uint32_t *words, int64_t n, hipStream_t s) {
  for (int64_t o = 0; o < n; o += kWordBlock) {
    WordBlock blk;
    const int m = int(n - o < kWordBlock ? n - o : kWordBlock);
    for (int i = 0; i < m; ++i) blk.w[i] = words[o + i];
    hipLaunchKernelGGL(write_words_kernel, dim3(1), dim3(256), 0, s, dst + o, blk, m);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t launch_cfl<PrecF64>(const PatchDev *, const int32_t *, int32_t, int32_t,
                                        int32_t, int32_t, const Params &, unsigned long long *,
                                        double *, hipStream_t);
template hipError_t launch_cfl<PrecMixed>(const PatchDev *, const int32_t *, int32_t, int32_t,
                                          int32_t, int32_t, const Params &, unsigned long long *,
                                          double *, hipStream_t);
template hipError_t launch_expansion<PrecF64>(const PatchDev *, const int32_t *, int32_t, int32_t,
                                              int32_t, double, const double *, const double *,
                                              hipStream_t);
template hipError_t launch_expansion<PrecMixed>(const PatchDev *, const int32_t *, int32_t,
                                                int32_t, int32_t, double, const double *,
                                                const double *, hipStream_t);
#define PPM_INSTANTIATE_AMR(Prec)                                                              \
  template hipError_t launch_capture<Prec>(const PatchDev *, const CaptureRow *, int32_t, int32_t, \
                                           const double *, const Params &, hipStream_t);        \
  template hipError_t launch_flux_correct<Prec>(const PatchDev *, const CorrTarget *, int32_t,   \
                                                const CorrContrib *, const Params &,             \
                                                hipStream_t);                                    \
  template hipError_t launch_project<Prec>(const PatchDev *, const ProjItem *, const int64_t *,  \
                                           int32_t, int64_t, hipStream_t);
PPM_INSTANTIATE_AMR(PrecF64)
PPM_INSTANTIATE_AMR(PrecMixed)
#undef PPM_INSTANTIATE_AMR
template hipError_t launch_fill<PrecF64>(const PatchDev &, hipStream_t);
template hipError_t launch_fill<PrecMixed>(const PatchDev &, hipStream_t);
template hipError_t launch_fill_boundary<PrecF64>(const PatchDev &, const FaceRules &,
                                                  hipStream_t);
template hipError_t launch_fill_from_parent<PrecF64>(const PatchDev *, const InterpItem *,
                                                     const int64_t *, int32_t, int64_t,
                                                     const PatchDev *, hipStream_t);
template hipError_t launch_fill_from_parent<PrecMixed>(const PatchDev *, const InterpItem *,
                                                       const int64_t *, int32_t, int64_t,
                                                       const PatchDev *, hipStream_t);
template hipError_t launch_box_state<PrecF64>(const PatchDev *, const PatchDev *,
                                              const PatchDev *, const CellBox *, const int64_t *,
                                              int32_t, int64_t, bool, double, hipStream_t);
template hipError_t launch_box_state<PrecMixed>(const PatchDev *, const PatchDev *,
                                                const PatchDev *, const CellBox *,
                                                const int64_t *, int32_t, int64_t, bool, double,
                                                hipStream_t);
template hipError_t launch_copy_from_siblings<PrecF64>(const PatchDev *, const SiblingBox *,
                                                       const int64_t *, int32_t, int64_t,
                                                       hipStream_t);
template hipError_t launch_copy_from_siblings<PrecMixed>(const PatchDev *, const SiblingBox *,
                                                         const int64_t *, int32_t, int64_t,
                                                         hipStream_t);
template hipError_t launch_fill_boundary<PrecMixed>(const PatchDev &, const FaceRules &,
                                                    hipStream_t);
#endif  // PPM_PASS_FP64

}  // namespace ppm
