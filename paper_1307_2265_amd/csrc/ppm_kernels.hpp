// ppm_kernels.hpp -- launcher declarations shared by the kernels and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "ppm_sweep.hpp"

namespace ppm {

constexpr int kMaxBlock = 256;

template <class Prec>
hipError_t launch_sweep(const PatchDev *patches, const int32_t *chunk_start, int32_t npatch,
                        int32_t nblocks, int32_t block, int32_t axis, int32_t mask,
                        const double *dt_dev, const Params &P, unsigned long long *counters,
                        unsigned long long *smax_bits, const int32_t *groups, int32_t ngroups,
                        hipStream_t s, double *defer = nullptr);

// groups (nullable): the marching sweep numbers the pencils of runs of
// equal-length patches consecutively (layout in ppm_kernels.hip).
// defer (nullable; a plan of one patch, no groups): sweep_split_kernel, two
// threads per pencil, nblocks covering two threads per pencil, `defer` 30
// doubles per pencil of workspace.
// Lane-parallel variant (a wavefront streams a run of pencils); block = 64 * waves.
// smax_bits (nullable) of a sweep launch: the sweep is the last of its step and
// also takes the max signal speed per level of the cells it writes.
template <class Prec>
hipError_t launch_sweep_lanes(const PatchDev *patches, const int32_t *chunk_start, int32_t npatch,
                              int32_t nblocks, int32_t block, int32_t axis, int32_t mask,
                              const double *dt_dev, const Params &P,
                              unsigned long long *counters, unsigned long long *smax_bits,
                              hipStream_t s);

// The pencils of one patch from `pencil0` on, one per wavefront of the
// lane-parallel code (block = 64 * waves): the rest of a marching sweep.
template <class Prec>
hipError_t launch_sweep_tail(const PatchDev *patches, const int32_t *chunk_start, int32_t nblocks,
                             int32_t block, int32_t axis, int32_t mask, int32_t pencil0,
                             const double *dt_dev, const Params &P, unsigned long long *counters,
                             unsigned long long *smax_bits, hipStream_t s);

// Persistent batch kernel: the whole step of every patch in one launch.
template <class Prec>
hipError_t launch_batch(const PatchDev *patches, const int32_t *order, int32_t npatch,
                        int32_t nblocks, int32_t block, int32_t sweep_order, int32_t lanes_mask,
                        const double *dt_dev, const Params &P, unsigned long long *counters,
                        unsigned int *queue, unsigned long long *smax_bits, hipStream_t s);

// dt_dev[l] = cfl a_l / max signal speed of level l (+inf if none), a_l from
// expand (nullable: a = 1); clears the maxima.
hipError_t launch_cfl_finalize(int32_t nlevels, double cfl, const double *expand,
                               unsigned long long *smax_bits, double *dt_dev, hipStream_t s);

template <class Prec>
hipError_t launch_cfl(const PatchDev *patches, const int32_t *chunk_start, int32_t npatch,
                      int32_t nblocks, int32_t cells_per_block, int32_t nlevels, const Params &P,
                      unsigned long long *smax_bits, double *dt_dev, hipStream_t s);

// Expansion terms of the comoving equations over every patch's active cells
// (chunked like launch_cfl); expand: per level (a, adot), not null.
template <class Prec>
hipError_t launch_expansion(const PatchDev *patches, const int32_t *chunk_start, int32_t npatch,
                            int32_t nblocks, int32_t cells_per_block, double gamma,
                            const double *expand, const double *dt_dev, hipStream_t s);

template <class Prec>
hipError_t launch_fill(const PatchDev &pd, hipStream_t s);

// Domain boundary conditions of the six faces (-x,+x,-y,+y,-z,+z) of a patch,
// and the values of inflow faces (rho, vx, vy, vz, etot, eint).
enum : int32_t { kFacePeriodic = 0, kFaceReflecting = 1, kFaceOutflow = 2, kFaceInflow = 3 };
struct FaceRules {
  int32_t kind[6];
  double inflow[6][6];
};

// Ghost fill of one patch by per-face boundary conditions.
template <class Prec>
hipError_t launch_fill_boundary(const PatchDev &pd, const FaceRules &fr, hipStream_t s);

// A box of a patch's ghost cells that take their values from its parent:
// indices into the patch table, refinement factor, global start of the first
// active cell of the patch (in its level) and of its parent (in the parent's
// level), and the box [lo, hi) in the patch's local (ghosted) indices.
struct InterpItem {
  int32_t patch, parent, r;
  int32_t start[3], pstart[3];
  int32_t lo[3], hi[3];
};
// Cells of patch dst outside its active region that lie in the active
// region of sibling src: the box [lo, hi) in dst's local (ghosted) indices,
// and the offset from dst-local to src-local indices.
struct SiblingBox {
  int32_t dst, src;
  int32_t lo[3], hi[3], shift[3];
};

// Ghost cells of items[0..nitems): SecondOrderA interpolation of the parent's
// conserved quantities.  prefix[i] = first parent cell of item i in the launch
// (prefix[nitems] = total), an item counting the parent cells that its box's
// cells refine.  parent_tab (nullable): a patch table to read the parents'
// states from instead of `patches` (the parents blended in time).
template <class Prec>
hipError_t launch_fill_from_parent(const PatchDev *patches, const InterpItem *items,
                                   const int64_t *prefix, int32_t nitems, int64_t total,
                                   const PatchDev *parent_tab, hipStream_t s);

// A box [lo, hi) of one patch's local (ghosted) cells.
struct CellBox {
  int32_t patch;
  int32_t lo[3], hi[3];
  int32_t pad;
};

// Over the cells of boxes[0..nboxes) (prefix over their volumes), in all six
// fields of the patch tables, which share dimensions and differ in their
// field pointers: blend false, old <- cur (a parent's state saved before its
// step); blend true, mid <- (1 - w) old + w cur evaluated in double (the
// parent at a time between its last two states).
template <class Prec>
hipError_t launch_box_state(const PatchDev *cur, const PatchDev *old, const PatchDev *mid,
                            const CellBox *boxes, const int64_t *prefix, int32_t nboxes,
                            int64_t total, bool blend, double w, hipStream_t s);

// A face whose flux a coarse step records: the pencil (i1, i2) of `patch`
// along the capture launch's axis, the face between its cells j and j+1
// (ghosted indices), and where dt F goes: dst[lab * fstride] for the six lab
// quantities.
struct CaptureRow {
  int32_t patch, i1, i2, j;
  double *dst;
  int64_t fstride;
};

// Final fluxes of rows[0..nrows) from the current state (the input of the
// sweep along `axis` that follows), six rows per wavefront.
template <class Prec>
hipError_t launch_capture(const PatchDev *patches, const CaptureRow *rows, int32_t nrows,
                          int32_t axis, const double *dt_dev, const Params &P, hipStream_t s);

// acc[i] += reg[i] over the listed register blocks (prefix over their sizes).
struct AccItem {
  double *acc;
  const double *reg;
};
hipError_t launch_accumulate(const AccItem *items, const int64_t *prefix, int32_t nitems,
                             int64_t total, hipStream_t s);

// Flux correction: one coarse cell per target, its contributions applied in
// list order.  A contribution is one face of a child footprint: the coarse
// dt F of the face (cap[k * cap_fstride]) and the r x r fine accumulated
// fluxes (fine[k * fine_fstride + jj * fine_row + ii]).
struct CorrTarget {
  int32_t patch, first, count, pad;
  int64_t cell;
};
struct CorrContrib {
  const double *cap;
  const double *fine;
  int64_t cap_fstride, fine_fstride;
  int32_t fine_row, r, side, axis;
};
template <class Prec>
hipError_t launch_flux_correct(const PatchDev *patches, const CorrTarget *targets,
                               int32_t ntargets, const CorrContrib *contribs, const Params &P,
                               hipStream_t s);

// Projection of children onto the coarse cells of their footprints (boxes in
// the coarse patch's active-local cells); prefix over box volumes.
struct ProjItem {
  int32_t coarse, fine, r, pad;
  int32_t lo[3], hi[3];
};
template <class Prec>
hipError_t launch_project(const PatchDev *patches, const ProjItem *items, const int64_t *prefix,
                          int32_t nitems, int64_t total, hipStream_t s);

// Sibling copies of boxes[0..nboxes); prefix as above, over box volumes.
template <class Prec>
hipError_t launch_copy_from_siblings(const PatchDev *patches, const SiblingBox *boxes,
                                     const int64_t *prefix, int32_t nboxes, int64_t total,
                                     hipStream_t s);

// quot[i] = ddiv(a[i], b[i]) and root[i] = dsqrt(a[i]) over n elements: the
// correctly rounded FP64 division and square root of the sweeps, exposed so
// that they can be checked against host IEEE arithmetic.
hipError_t launch_fp64_ops(const double *a, const double *b, double *quot, double *root,
                           int64_t n, hipStream_t s);

// dst[i] = words[i] for i < n (32-bit words from host memory, carried to the
// device as kernel arguments, so no staging copy and no memset is involved).
hipError_t launch_write_words(uint32_t *dst, const uint32_t *words, int64_t n, hipStream_t s);

}  // namespace ppm
