// ppm_plan.hpp -- the plan behind the C ABI's opaque ppm_plan, and the
// library-internal helpers the ABI's source files share.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "ppm.h"
#include "ppm_kernels.hpp"

using ppm::PatchDev;

struct ppm_plan {
  int32_t npatch = 0, nlevels = 0;
  ppm_precision prec = PPM_FP64;
  ppm::Params P{};
  int32_t block = 256;            // threads (pencils) per marching-sweep block
  int32_t lanes_block = 256;      // threads per lane-parallel block (64 per pencil)
  int32_t lanes_mask = 1;         // bit a: sweeps along axis a use the lane-parallel kernel
  bool lanes_set = false;         // lanes, or a marching-sweep shape, given in the tile config
  int32_t cfl_cells = 4096;       // active cells per CFL block
  int32_t persistent = 0;         // ppm_step as one persistent launch over all patches
  int32_t batch_block = 256;      // threads per workgroup of the persistent kernel
  int32_t batch_blocks = 0;       // workgroups of the persistent kernel
  int32_t group = 0;              // marching sweeps number pencils across equal-length patches
  bool group_set = false;         // group given in the tile config
  int32_t tail = 1;               // one patch: lanes launch for a marching sweep's last round
  int32_t tail_round = 0;         // pencils per marching round (0: from the occupancy)
  int32_t tail_pencil0[2][12] = {};  // [cfl][slot]: first pencil of the lanes tail
  int32_t tail_main[2][12] = {};     // marching blocks before it
  int32_t tail_blocks[2][12] = {};   // lane-parallel blocks of the tail (0: no tail)
  int32_t split = 1;              // one patch, few pencils: two threads march each pencil
  int32_t split_on[2][12] = {};   // [cfl][slot]: this marching sweep is split
  int32_t split_blocks[2][12] = {};  // its marching blocks when there is no tail
  double *d_defer = nullptr;      // split marching: 30 doubles per pencil
  int32_t *d_order = nullptr;     // patches by descending cost (persistent queue order)
  unsigned int *d_queue = nullptr;  // persistent queue head and exit count
  std::vector<PatchDev> host;
  std::vector<int32_t> bc;        // boundary kind of each patch
  PatchDev *d_patches = nullptr;
  int32_t *d_chunks = nullptr;    // 12 marching, 12 lane-parallel prefix arrays, then CFL
  int32_t nblocks[24] = {};
  int32_t *d_groups = nullptr;    // grouped marching maps of the 12 (axis, extent) slots
  int64_t gofs[12] = {};          // offset of each slot's map in d_groups
  int32_t ngroups[12] = {};
  int32_t cfl_blocks = 0;
  unsigned long long *d_counters = nullptr;  // fallback faces, floored cells
  unsigned long long *d_smax = nullptr;      // per-level max signal speed bits
  int device = 0;
  // AMR ghost fill work lists, grouped by level (ppm_set_hierarchy)
  bool hier = false;
  std::vector<ppm::InterpItem> h_interp;  // host copy of the interpolation boxes
  ppm::InterpItem *d_interp = nullptr;
  ppm::SiblingBox *d_boxes = nullptr;
  int64_t *d_iprefix = nullptr, *d_bprefix = nullptr;  // per level: items+1 / boxes+1 entries
  std::vector<int32_t> ibeg, bbeg;        // per level: first item / box (nlevels+1 entries)
  std::vector<int64_t> itotal, btotal;    // per level: parent cells / box cells
};

namespace ppm_detail {

// Record the error message of the last failing call (ppm_last_error) and
// return s.
ppm_status fail(ppm_status s, const char *fmt, ...);
ppm_status hip_fail(hipError_t e, const char *what);

// Argument checks shared by the entry points (PPM_EINVAL with a message).
ppm_status check_params(const ppm_params *p);
ppm_status check_patch(const ppm_patch &q, int i, int32_t nlevels);
// PPM_MIXED: rho_floor and p_floor must be normal floats.
ppm_status check_mixed_floors(ppm_precision prec, const ppm_params *p);
// The smallest float not below x (x a positive double in the float range).
double float_at_or_above(double x);
// The device parameters of a precision (PPM_MIXED floors raised to floats;
// no expansion factors).
ppm::Params device_params(ppm_precision prec, const ppm_params *p);

// A box [lo, hi) of cell indices.
struct IBox {
  int64_t lo[3], hi[3];
  int64_t volume() const { return (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]); }
};
// Replace the boxes of `list` by their parts outside b: each box that meets b
// splits into at most six disjoint pieces, so disjoint boxes stay disjoint.
void boxes_minus(std::vector<IBox> &list, const IBox &b);

// ppm_fill_ghosts of `level`, with the parents' states read through
// parent_tab (a device patch table in the plan's order) when it is given.
ppm_status fill_ghosts(ppm_plan *plan, int32_t level, const PatchDev *parent_tab, hipStream_t s);

}  // namespace ppm_detail
