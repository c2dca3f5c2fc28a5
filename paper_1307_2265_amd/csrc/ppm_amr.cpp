// ppm_amr.cpp -- the AMR level step on a static hierarchy (ppm_amr_* in
// include/ppm.h).
//
// The W-cycle of Sec. "Adaptive Mesh Refinement" (EvolveLevel) over a fixed
// patch tree: each level is a plan of its own (its sweeps, CFL reductions and
// launch maps), and one plan over every patch carries the hierarchy's ghost
// fill.  The host keeps the level times and takes each level's timestep from
// the device (one small copy per level step), so the number of substeps is
// known where the recursion runs; everything else stays on the device.  The
// work lists of the coarse-fine coupling -- the faces whose coarse fluxes a
// step records, the registers summed over substeps, the corrected coarse
// cells with their contributions in order, the projected coarse cells -- are
// built here once, from the same loops the oracle runs, so the device applies
// the same operations in the same order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>

#include "ppm.h"
#include "ppm_kernels.hpp"
#include "ppm_plan.hpp"

using ppm_detail::fail;
using ppm_detail::hip_fail;

namespace {

const int kAmrOrders[2][3] = {{0, 1, 2}, {2, 1, 0}};

int64_t reg_face_offset(int64_t nx, int64_t ny, int64_t nz, int face) {
  const int64_t area[3] = {ny * nz, nx * nz, nx * ny};
  int64_t off = 0;
  for (int f = 0; f < face; ++f) off += 6 * area[f / 2];
  return off;
}

struct Box {
  int32_t lo[3], hi[3];
  bool has(int x, int y, int z) const {
    return x >= lo[0] && x < hi[0] && y >= lo[1] && y < hi[1] && z >= lo[2] && z < hi[2];
  }
  int64_t dim(int a) const { return int64_t(hi[a]) - lo[a]; }
};

template <class T> hipError_t upload(T **dst, const std::vector<T> &v) {
  *dst = nullptr;
  if (v.empty()) return hipSuccess;
  hipError_t e = hipMalloc(dst, sizeof(T) * v.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

}  // namespace

struct ppm_amr {
  int32_t npatch = 0, nlevels = 0;
  ppm_precision prec = PPM_FP64;
  std::vector<ppm_patch> patches;
  std::vector<ppm_patch_place> place;
  std::vector<std::vector<int32_t>> members;   // per level: patch indices
  std::vector<std::vector<int32_t>> children;  // per patch: child indices
  std::vector<Box> footprint;                  // per child: its box in the parent
  ppm_plan *all = nullptr;                     // every patch: ghost fill
  std::vector<ppm_plan *> lplan;               // per level
  bool root_periodic = true;
  int32_t root_kinds[6] = {};
  double root_inflow[36] = {};
  bool has_inflow = false;
  double *d_dt = nullptr, *d_cfl = nullptr;    // nlevels doubles each
  double h_dt[64] = {}, h_cfl = 0.0;
  // parents' states before their last step, and blended to a child's time
  std::vector<void *> old_bufs, blend_bufs;
  PatchDev *d_old = nullptr;                   // patch tables with the saved states and
  PatchDev *d_blend = nullptr;                 // the blends of the parents
  // per parent level: the parent cells its children's interpolation reads
  ppm::CellBox *d_need = nullptr;
  int64_t *d_needprefix = nullptr;             // one extra entry per level
  std::vector<int32_t> need_beg;               // nlevels + 1
  std::vector<int64_t> need_total;
  // coarse fluxes through child footprints, per level and axis
  double *d_cap = nullptr;
  ppm::CaptureRow *d_rows = nullptr;
  std::vector<int64_t> row_beg;                // [level * 3 + axis] .. +1
  // fine registers summed over substeps
  double *d_acc = nullptr;
  std::vector<int64_t> acc_off;                // per patch (-1 on the root)
  ppm::AccItem *d_accitems = nullptr;
  int64_t *d_accprefix = nullptr;
  std::vector<int32_t> acc_beg;                // per level: first item (nlevels + 1)
  std::vector<int64_t> acc_total;              // per level: values summed
  std::vector<int64_t> acc_span;               // per level: its registers' whole block
  // flux correction, per coarse level
  ppm::CorrTarget *d_targets = nullptr;
  ppm::CorrContrib *d_contribs = nullptr;
  std::vector<int32_t> tgt_beg;                // nlevels + 1
  // projection, per child level
  ppm::ProjItem *d_proj = nullptr;
  int64_t *d_projprefix = nullptr;
  std::vector<int32_t> proj_beg;               // nlevels + 1
  std::vector<int64_t> proj_total;
  // level times
  std::vector<double> t, t_old;
  std::vector<int64_t> nsteps;
  std::vector<char> stepped;
  std::vector<std::pair<int32_t, double>> log; // (level, dt) since the last ppm_amr_step
  const double *expand = nullptr;              // per-level a, adot (ppm_amr_set_expansion)
};

namespace {

void destroy(ppm_amr *h) {
  if (!h) return;
  if (h->all) ppm_plan_destroy(h->all);
  for (ppm_plan *p : h->lplan)
    if (p) ppm_plan_destroy(p);
  for (void *b : h->old_bufs) (void)hipFree(b);
  for (void *b : h->blend_bufs) (void)hipFree(b);
  void *bufs[] = {h->d_dt,   h->d_cfl,      h->d_old,       h->d_blend,   h->d_cap,
                  h->d_rows, h->d_acc,      h->d_accitems,  h->d_accprefix, h->d_targets,
                  h->d_contribs, h->d_proj, h->d_projprefix, h->d_need,   h->d_needprefix};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  delete h;
}

size_t storage_bytes(ppm_precision prec) { return prec == PPM_FP64 ? 8 : 4; }

int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

int64_t ghosted_cells(const ppm_patch &q) {
  return (int64_t(q.nx) + 2 * q.ghost) * (int64_t(q.ny) + 2 * q.ghost) *
         (int64_t(q.nz) + 2 * q.ghost);
}

// ---- the steps of EvolveLevel ----------------------------------------------

ppm_status fill(ppm_amr *h, int l, hipStream_t s) {
  if (l == 0) {
    if (h->root_periodic) return ppm_fill_periodic(h->lplan[0], s);
    return ppm_fill_boundary(h->lplan[0], 0, h->root_kinds,
                             h->has_inflow ? h->root_inflow : nullptr, s);
  }
  const int pl = l - 1;
  if (!(h->t[pl] != h->t_old[pl] && h->stepped[pl]))
    return ppm_detail::fill_ghosts(h->all, l, nullptr, s);
  // the parents' stored fields at this level's time, blended in double
  const double w = (h->t[l] - h->t_old[pl]) / (h->t[pl] - h->t_old[pl]);
  const int32_t b0 = h->need_beg[pl], nb = h->need_beg[pl + 1] - b0;
  hipError_t e = h->prec == PPM_FP64
      ? ppm::launch_box_state<ppm::PrecF64>(h->all->d_patches, h->d_old, h->d_blend,
                                            h->d_need + b0, h->d_needprefix + b0 + pl, nb,
                                            h->need_total[pl], true, w, s)
      : ppm::launch_box_state<ppm::PrecMixed>(h->all->d_patches, h->d_old, h->d_blend,
                                              h->d_need + b0, h->d_needprefix + b0 + pl, nb,
                                              h->need_total[pl], true, w, s);
  if (e != hipSuccess) return hip_fail(e, "time blend launch");
  return ppm_detail::fill_ghosts(h->all, l, h->d_blend, s);
}

ppm_status level_dt(ppm_amr *h, int l, hipStream_t s, double *dt) {
  ppm_status st = ppm_cfl_dt(h->lplan[l], h->d_cfl, s);
  if (st != PPM_OK) return st;
  hipError_t e = hipMemcpyAsync(&h->h_cfl, h->d_cfl + l, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "level timestep");
  *dt = h->h_cfl;
  if (!(*dt > 0.0) || !(*dt < __builtin_inf()))
    return fail(PPM_EINVAL, "level %d: no finite positive CFL timestep", l);
  return PPM_OK;
}

ppm_status step_level(ppm_amr *h, int l, int order, hipStream_t s) {
  const bool capture = h->row_beg[l * 3 + 3] > h->row_beg[l * 3];
  if (!capture) return ppm_step(h->lplan[l], h->d_dt, order, s);
  int mask = 0;
  for (int k = 0; k < 3; ++k) {
    const int axis = kAmrOrders[order][k];
    const int64_t r0 = h->row_beg[l * 3 + axis], r1 = h->row_beg[l * 3 + axis + 1];
    hipError_t e = h->prec == PPM_FP64
        ? ppm::launch_capture<ppm::PrecF64>(h->all->d_patches, h->d_rows + r0, int32_t(r1 - r0),
                                            axis, h->d_dt, h->lplan[l]->P, s)
        : ppm::launch_capture<ppm::PrecMixed>(h->all->d_patches, h->d_rows + r0,
                                              int32_t(r1 - r0), axis, h->d_dt, h->lplan[l]->P, s);
    if (e != hipSuccess) return hip_fail(e, "capture launch");
    ppm_status st = ppm_sweep(h->lplan[l], h->d_dt, axis, mask, s);
    if (st != PPM_OK) return st;
    mask |= 1 << axis;
  }
  return PPM_OK;
}

ppm_status save_old(ppm_amr *h, int l, hipStream_t s) {
  const int32_t b0 = h->need_beg[l], nb = h->need_beg[l + 1] - b0;
  if (nb == 0) return PPM_OK;
  hipError_t e = h->prec == PPM_FP64
      ? ppm::launch_box_state<ppm::PrecF64>(h->all->d_patches, h->d_old, h->d_blend,
                                            h->d_need + b0, h->d_needprefix + b0 + l, nb,
                                            h->need_total[l], false, 0.0, s)
      : ppm::launch_box_state<ppm::PrecMixed>(h->all->d_patches, h->d_old, h->d_blend,
                                              h->d_need + b0, h->d_needprefix + b0 + l, nb,
                                              h->need_total[l], false, 0.0, s);
  if (e != hipSuccess) return hip_fail(e, "old-state copy launch");
  return PPM_OK;
}

ppm_status correct_and_project(ppm_amr *h, int l, hipStream_t s) {
  hipError_t e;
  const int32_t t0 = h->tgt_beg[l], nt = h->tgt_beg[l + 1] - t0;
  if (nt > 0) {
    e = h->prec == PPM_FP64
        ? ppm::launch_flux_correct<ppm::PrecF64>(h->all->d_patches, h->d_targets + t0, nt,
                                                 h->d_contribs, h->lplan[l]->P, s)
        : ppm::launch_flux_correct<ppm::PrecMixed>(h->all->d_patches, h->d_targets + t0, nt,
                                                   h->d_contribs, h->lplan[l]->P, s);
    if (e != hipSuccess) return hip_fail(e, "flux correction launch");
  }
  // the children's sums start again for the next step of this level
  const int c = l + 1;
  if (h->acc_total[c] > 0) {
    const int64_t first = h->acc_off[h->members[c].front()];
    e = hipMemsetAsync(h->d_acc + first, 0, sizeof(double) * size_t(h->acc_span[c]), s);
    if (e != hipSuccess) return hip_fail(e, "register sums reset");
  }
  const int32_t p0 = h->proj_beg[c], np = h->proj_beg[c + 1] - p0;
  if (np > 0) {
    const int64_t *pp = h->d_projprefix + p0 + c;
    e = h->prec == PPM_FP64
        ? ppm::launch_project<ppm::PrecF64>(h->all->d_patches, h->d_proj + p0, pp, np,
                                            h->proj_total[c], s)
        : ppm::launch_project<ppm::PrecMixed>(h->all->d_patches, h->d_proj + p0, pp, np,
                                              h->proj_total[c], s);
    if (e != hipSuccess) return hip_fail(e, "projection launch");
  }
  return PPM_OK;
}

ppm_status evolve(ppm_amr *h, int l, double t_end, bool has_end, hipStream_t s) {
  ppm_status st = fill(h, l, s);
  if (st != PPM_OK) return st;
  while (!has_end || h->t[l] < t_end) {
    double dt;
    if ((st = level_dt(h, l, s, &dt)) != PPM_OK) return st;
    double t_new = h->t[l] + dt;
    if (has_end && dt >= t_end - h->t[l]) {
      dt = t_end - h->t[l];
      t_new = t_end;
    }
    h->log.emplace_back(l, dt);
    h->h_dt[l] = dt;
    hipError_t e = hipMemcpyAsync(h->d_dt + l, &h->h_dt[l], sizeof(double),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "level timestep upload");
    const int order = int(h->nsteps[l] % 2);
    if ((st = save_old(h, l, s)) != PPM_OK) return st;
    if ((st = step_level(h, l, order, s)) != PPM_OK) return st;
    if (l > 0 && h->acc_total[l] > 0) {
      const int32_t i0 = h->acc_beg[l], ni = h->acc_beg[l + 1] - i0;
      e = ppm::launch_accumulate(h->d_accitems + i0, h->d_accprefix + i0 + l, ni,
                                 h->acc_total[l], s);
      if (e != hipSuccess) return hip_fail(e, "register sum launch");
    }
    if (h->expand && (st = ppm_expansion(h->lplan[l], h->d_dt, s)) != PPM_OK) return st;
    h->t_old[l] = h->t[l];
    h->t[l] = t_new;
    h->nsteps[l] += 1;
    h->stepped[l] = 1;
    if ((st = fill(h, l, s)) != PPM_OK) return st;
    if (l + 1 < h->nlevels && !h->members[l + 1].empty()) {
      if ((st = evolve(h, l + 1, h->t[l], true, s)) != PPM_OK) return st;
      if ((st = correct_and_project(h, l, s)) != PPM_OK) return st;
    }
    if (!has_end) break;
  }
  return PPM_OK;
}

// ---- set-up ------------------------------------------------------------------

ppm_status build_lists(ppm_amr *h) {
  const int L = h->nlevels, np = h->npatch;
  const size_t sb = storage_bytes(h->prec);
  hipError_t e;
  // old-state and blend buffers of every patch with children, and the patch
  // tables through which the saves and blends write them and the parent
  // interpolation reads the blends
  h->old_bufs.assign(size_t(np) * 6, nullptr);
  h->blend_bufs.assign(size_t(np) * 6, nullptr);
  std::vector<PatchDev> old_tab(h->all->host), blend_tab(h->all->host);
  for (int p = 0; p < np; ++p) {
    if (h->children[p].empty()) continue;
    const int64_t n = ghosted_cells(h->patches[p]);
    for (int f = 0; f < 6; ++f) {
      const size_t bytes = size_t(n) * (f < 4 ? sb : 8);
      if ((e = hipMalloc(&h->old_bufs[size_t(p) * 6 + f], bytes)) != hipSuccess ||
          (e = hipMalloc(&h->blend_bufs[size_t(p) * 6 + f], bytes)) != hipSuccess)
        return hip_fail(e, "old-state allocation");
    }
    for (int k = 0; k < 2; ++k) {
      PatchDev &d = k ? blend_tab[p] : old_tab[p];
      const std::vector<void *> &bufs = k ? h->blend_bufs : h->old_bufs;
      d.rho = bufs[size_t(p) * 6];
      for (int a = 0; a < 3; ++a) d.vel[a] = bufs[size_t(p) * 6 + 1 + a];
      d.etot = static_cast<double *>(bufs[size_t(p) * 6 + 4]);
      d.eint = static_cast<double *>(bufs[size_t(p) * 6 + 5]);
    }
  }
  if ((e = upload(&h->d_old, old_tab)) != hipSuccess ||
      (e = upload(&h->d_blend, blend_tab)) != hipSuccess)
    return hip_fail(e, "saved-state tables");
  // The parent cells that the children's ghost interpolation reads: the
  // 27-cell neighbourhoods of the parent cells that its boxes refine, merged
  // per parent into disjoint boxes.  Only these cells are saved before a
  // parent's step and blended to a child's time.
  {
    std::vector<std::vector<ppm_detail::IBox>> need(static_cast<size_t>(np));
    const ppm_plan *A = h->all;
    for (const ppm::InterpItem &it : A->h_interp) {
      const PatchDev &f = A->host[it.patch], &c = A->host[it.parent];
      ppm_detail::IBox b{};
      for (int a = 0; a < 3; ++a) {
        const int64_t c0 = floor_div(int64_t(it.start[a]) + it.lo[a] - f.ghost, it.r);
        const int64_t c1 = floor_div(int64_t(it.start[a]) + it.hi[a] - 1 - f.ghost, it.r);
        b.lo[a] = c0 - 1 - it.pstart[a] + c.ghost;
        b.hi[a] = c1 + 2 - it.pstart[a] + c.ghost;
      }
      std::vector<ppm_detail::IBox> pieces{b};
      for (const ppm_detail::IBox &q : need[size_t(it.parent)]) ppm_detail::boxes_minus(pieces, q);
      need[size_t(it.parent)].insert(need[size_t(it.parent)].end(), pieces.begin(), pieces.end());
    }
    std::vector<ppm::CellBox> boxes;
    std::vector<int64_t> prefix;
    h->need_beg.assign(size_t(L) + 1, 0);
    h->need_total.assign(size_t(L) + 1, 0);
    for (int l = 0; l < L; ++l) {
      h->need_beg[l] = int32_t(boxes.size());
      int64_t run = 0;
      for (int32_t p : h->members[l])
        for (const ppm_detail::IBox &q : need[size_t(p)]) {
          ppm::CellBox cb{};
          cb.patch = p;
          for (int a = 0; a < 3; ++a) {
            cb.lo[a] = int32_t(q.lo[a]);
            cb.hi[a] = int32_t(q.hi[a]);
          }
          boxes.push_back(cb);
          prefix.push_back(run);
          run += q.volume();
        }
      prefix.push_back(run);
      h->need_total[l] = run;
    }
    h->need_beg[L] = int32_t(boxes.size());
    if ((e = upload(&h->d_need, boxes)) != hipSuccess ||
        (e = upload(&h->d_needprefix, prefix)) != hipSuccess)
      return hip_fail(e, "saved-cell lists");
  }

  // The coarse cell next to face `face` of child c's footprint at transverse
  // position (c1, c2) of the face, in the parent's active-cell indices, and
  // whether flux correction uses it: only where no child of the parent
  // covers that coarse cell does the coarse flux through the face meet the
  // fine fluxes (elsewhere both sides are fine cells).
  auto face_cell = [&](int32_t c, int face, int c1, int c2, int cc[3]) {
    const Box &b = h->footprint[c];
    const int a = face / 2, side = face % 2;
    const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
    cc[a] = side == 0 ? b.lo[a] - 1 : b.hi[a];
    cc[t1] = b.lo[t1] + c1;
    cc[t2] = b.lo[t2] + c2;
    bool covered = false;
    for (int32_t o : h->children[h->place[c].parent])
      covered = covered || h->footprint[o].has(cc[0], cc[1], cc[2]);
    return !covered;
  };
  // faces of each child that some correction reads
  std::vector<std::array<bool, 6>> face_used(static_cast<size_t>(np));
  for (int c = 0; c < np; ++c) {
    face_used[size_t(c)].fill(false);
    if (h->place[c].parent < 0) continue;
    const Box &b = h->footprint[c];
    for (int face = 0; face < 6; ++face) {
      const int a = face / 2;
      const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
      int cc[3];
      bool used = false;
      for (int c2 = 0; c2 < b.dim(t2) && !used; ++c2)
        for (int c1 = 0; c1 < b.dim(t1) && !used; ++c1) used = face_cell(c, face, c1, c2, cc);
      face_used[size_t(c)][size_t(face)] = used;
    }
  }

  // capture blocks: per parent, per child, a register-shaped block
  std::vector<int64_t> cap_off(size_t(np), -1);  // per child
  int64_t cap_total = 0;
  for (int p = 0; p < np; ++p)
    for (int32_t c : h->children[p]) {
      const Box &b = h->footprint[c];
      cap_off[c] = cap_total;
      cap_total += reg_face_offset(b.dim(0), b.dim(1), b.dim(2), 6);
    }
  if (cap_total > 0 && (e = hipMalloc(&h->d_cap, sizeof(double) * size_t(cap_total))) != hipSuccess)
    return hip_fail(e, "capture allocation");
  // fine register sums, contiguous per level
  h->acc_off.assign(size_t(np), -1);
  int64_t acc_total = 0;
  h->acc_beg.assign(size_t(L) + 1, 0);
  h->acc_total.assign(size_t(L) + 1, 0);
  h->acc_span.assign(size_t(L) + 1, 0);
  std::vector<int64_t> acc_item_off;       // offset of each item's sum in d_acc
  std::vector<const double *> acc_item_reg;
  std::vector<int64_t> accprefix;
  // (only the faces that a correction reads are summed)
  for (int l = 0; l < L; ++l) {
    h->acc_beg[l] = int32_t(acc_item_off.size());
    int64_t run = 0;
    for (int32_t p : h->members[l]) {
      if (l == 0) continue;
      const ppm_patch &q = h->patches[p];
      const int64_t n = ppm_flux_reg_size(q.nx, q.ny, q.nz);
      h->acc_off[p] = acc_total;
      for (int face = 0; face < 6; ++face) {
        if (!face_used[size_t(p)][size_t(face)]) continue;
        const int64_t f0 = reg_face_offset(q.nx, q.ny, q.nz, face);
        const int64_t f1 = reg_face_offset(q.nx, q.ny, q.nz, face + 1);
        acc_item_off.push_back(acc_total + f0);
        acc_item_reg.push_back(q.flux_reg + f0);
        accprefix.push_back(run);
        run += f1 - f0;
      }
      acc_total += n;
      h->acc_span[l] += n;
    }
    accprefix.push_back(run);
    h->acc_total[l] = run;
  }
  h->acc_beg[L] = int32_t(acc_item_off.size());
  if (acc_total > 0) {
    if ((e = hipMalloc(&h->d_acc, sizeof(double) * size_t(acc_total))) != hipSuccess ||
        (e = hipMemset(h->d_acc, 0, sizeof(double) * size_t(acc_total))) != hipSuccess)
      return hip_fail(e, "register sum allocation");
  }
  std::vector<ppm::AccItem> accitems;
  for (size_t i = 0; i < acc_item_off.size(); ++i)
    accitems.push_back(ppm::AccItem{h->d_acc + acc_item_off[i], acc_item_reg[i]});
  if ((e = upload(&h->d_accitems, accitems)) != hipSuccess ||
      (e = upload(&h->d_accprefix, accprefix)) != hipSuccess)
    return hip_fail(e, "register sum lists");

  // capture rows per (level, axis)
  std::vector<ppm::CaptureRow> rows;
  h->row_beg.assign(size_t(L) * 3 + 1, 0);
  for (int l = 0; l < L; ++l)
    for (int axis = 0; axis < 3; ++axis) {
      h->row_beg[size_t(l) * 3 + axis] = int64_t(rows.size());
      const int t1 = axis == 0 ? 1 : 0, t2 = axis == 2 ? 1 : 2;
      for (int32_t p : h->members[l]) {
        const int g = h->patches[p].ghost;
        for (int32_t c : h->children[p]) {
          const Box &b = h->footprint[c];
          const int64_t fs = b.dim(t1) * b.dim(t2);
          for (int side = 0; side < 2; ++side) {
            double *face = h->d_cap + cap_off[c] +
                           reg_face_offset(b.dim(0), b.dim(1), b.dim(2), 2 * axis + side);
            int cc[3];
            for (int c2 = 0; c2 < b.dim(t2); ++c2)
              for (int c1 = 0; c1 < b.dim(t1); ++c1)
                if (face_cell(c, 2 * axis + side, c1, c2, cc))
                  rows.push_back(ppm::CaptureRow{
                    p, g + b.lo[t1] + c1, g + b.lo[t2] + c2,
                    g + (side == 0 ? b.lo[axis] - 1 : b.hi[axis] - 1),
                    face + int64_t(c2) * b.dim(t1) + c1, fs});
          }
        }
      }
    }
  h->row_beg[size_t(L) * 3] = int64_t(rows.size());
  if ((e = upload(&h->d_rows, rows)) != hipSuccess) return hip_fail(e, "capture rows");

  // flux correction: per coarse cell, its contributions in box, face order
  std::vector<ppm::CorrTarget> targets;
  std::vector<ppm::CorrContrib> contribs;
  h->tgt_beg.assign(size_t(L) + 1, 0);
  for (int l = 0; l < L; ++l) {
    h->tgt_beg[l] = int32_t(targets.size());
    for (int32_t p : h->members[l]) {
      const auto &ch = h->children[p];
      if (ch.empty()) continue;
      const ppm_patch &q = h->patches[p];
      const int g = q.ghost;
      const int64_t n0 = int64_t(q.nx) + 2 * g, n1 = int64_t(q.ny) + 2 * g;
      std::map<int64_t, std::vector<ppm::CorrContrib>> per_cell;
      std::vector<int64_t> cell_order;
      for (int32_t c : ch) {
        const Box &b = h->footprint[c];
        const int r = h->place[c].refine;
        const int64_t fd[3] = {b.dim(0) * r, b.dim(1) * r, b.dim(2) * r};
        const double *acc = h->d_acc + h->acc_off[c];
        for (int face = 0; face < 6; ++face) {
          const int a = face / 2, side = face % 2;
          const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
          const double *cface = h->d_cap + cap_off[c] +
                                reg_face_offset(b.dim(0), b.dim(1), b.dim(2), face);
          const double *fface = acc + reg_face_offset(fd[0], fd[1], fd[2], face);
          for (int c2 = 0; c2 < b.dim(t2); ++c2)
            for (int c1 = 0; c1 < b.dim(t1); ++c1) {
              int cc[3];
              if (!face_cell(c, face, c1, c2, cc)) continue;
              const int64_t cell = ((int64_t(cc[2]) + g) * n1 + (cc[1] + g)) * n0 + (cc[0] + g);
              ppm::CorrContrib cb;
              cb.cap = cface + int64_t(c2) * b.dim(t1) + c1;
              cb.fine = fface + int64_t(c2) * r * fd[t1] + int64_t(c1) * r;
              cb.cap_fstride = b.dim(t1) * b.dim(t2);
              cb.fine_fstride = fd[t1] * fd[t2];
              cb.fine_row = int32_t(fd[t1]);
              cb.r = r;
              cb.side = side;
              cb.axis = a;
              auto it = per_cell.find(cell);
              if (it == per_cell.end()) {
                cell_order.push_back(cell);
                per_cell[cell] = {cb};
              } else {
                it->second.push_back(cb);
              }
            }
        }
      }
      for (int64_t cell : cell_order) {
        const auto &v = per_cell[cell];
        targets.push_back(ppm::CorrTarget{p, int32_t(contribs.size()), int32_t(v.size()), 0, cell});
        contribs.insert(contribs.end(), v.begin(), v.end());
      }
    }
  }
  h->tgt_beg[L] = int32_t(targets.size());
  if ((e = upload(&h->d_targets, targets)) != hipSuccess ||
      (e = upload(&h->d_contribs, contribs)) != hipSuccess)
    return hip_fail(e, "flux correction lists");

  // projection items per child level (prefix arrays with one extra entry per level)
  std::vector<ppm::ProjItem> proj;
  std::vector<int64_t> pprefix;
  h->proj_beg.assign(size_t(L) + 1, 0);
  h->proj_total.assign(size_t(L) + 1, 0);
  for (int l = 0; l < L; ++l) {
    h->proj_beg[l] = int32_t(proj.size());
    int64_t run = 0;
    for (int32_t c : h->members[l]) {
      if (l == 0) continue;
      const Box &b = h->footprint[c];
      ppm::ProjItem it{};
      it.coarse = h->place[c].parent;
      it.fine = c;
      it.r = h->place[c].refine;
      for (int a = 0; a < 3; ++a) {
        it.lo[a] = b.lo[a];
        it.hi[a] = b.hi[a];
      }
      proj.push_back(it);
      pprefix.push_back(run);
      run += b.dim(0) * b.dim(1) * b.dim(2);
    }
    pprefix.push_back(run);
    h->proj_total[l] = run;
  }
  h->proj_beg[L] = int32_t(proj.size());
  if ((e = upload(&h->d_proj, proj)) != hipSuccess ||
      (e = upload(&h->d_projprefix, pprefix)) != hipSuccess)
    return hip_fail(e, "projection lists");
  return PPM_OK;
}

}  // namespace

extern "C" {

ppm_status ppm_amr_create(ppm_amr **out, const ppm_patch *patches, const ppm_patch_place *place,
                          int32_t npatch, int32_t nlevels, ppm_precision prec,
                          const ppm_params *params, const int32_t *root_kinds,
                          const double *root_inflow, void *hip_stream) {
  if (!out) return fail(PPM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!patches || !place) return fail(PPM_EINVAL, "patches or place is NULL");
  if (npatch < 1 || nlevels < 1 || nlevels > 64)
    return fail(PPM_EINVAL, "need npatch >= 1 and nlevels in 1..64");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  ppm_amr *h = new (std::nothrow) ppm_amr();
  if (!h) return fail(PPM_ENOMEM, "host allocation failed");
  h->npatch = npatch;
  h->nlevels = nlevels;
  h->prec = prec;
  h->patches.assign(patches, patches + npatch);
  h->place.assign(place, place + npatch);
  h->members.assign(size_t(nlevels), {});
  h->children.assign(size_t(npatch), {});
  h->footprint.assign(size_t(npatch), Box{});
  auto bail = [&](ppm_status st) {
    destroy(h);
    return st;
  };
  for (int p = 0; p < npatch; ++p) {
    const ppm_patch &q = patches[p];
    if (q.level < 0 || q.level >= nlevels)
      return bail(fail(PPM_EINVAL, "patch %d: level %d outside [0, %d)", p, q.level, nlevels));
    h->members[q.level].push_back(p);
  }
  if (h->members[0].size() != 1 || place[h->members[0][0]].parent != -1)
    return bail(fail(PPM_EINVAL, "the hierarchy needs exactly one root patch on level 0"));
  for (int l = 1; l < nlevels; ++l)
    if (h->members[l].empty() && l + 1 < nlevels && !h->members[l + 1].empty())
      return bail(fail(PPM_EINVAL, "level %d is empty but a finer level is not", l));
  for (int p = 0; p < npatch; ++p) {
    const ppm_patch &q = patches[p];
    if (q.level == 0) continue;
    const int par = place[p].parent, r = place[p].refine;
    if (par < 0 || par >= npatch || patches[par].level != q.level - 1)
      return bail(fail(PPM_EINVAL, "patch %d: parent must be a patch one level coarser", p));
    if (!q.flux_reg)
      return bail(fail(PPM_EINVAL, "patch %d: patches below the root need flux registers", p));
    if (r < 2) return bail(fail(PPM_EINVAL, "patch %d: refinement factor must be >= 2", p));
    const int32_t dims[3] = {q.nx, q.ny, q.nz};
    const ppm_patch &pq = patches[par];
    const int32_t pd[3] = {pq.nx, pq.ny, pq.nz};
    Box b;
    for (int a = 0; a < 3; ++a) {
      if (place[p].start[a] % r != 0 || dims[a] % r != 0)
        return bail(fail(PPM_EINVAL, "patch %d: must start and end on parent cell boundaries", p));
      b.lo[a] = place[p].start[a] / r - place[par].start[a];
      b.hi[a] = b.lo[a] + dims[a] / r;
      if (b.lo[a] < 1 || b.hi[a] > pd[a] - 1)
        return bail(fail(PPM_EINVAL,
                         "patch %d: footprint must lie at least one cell inside the parent's "
                         "active region", p));
    }
    h->footprint[p] = b;
    for (int32_t o : h->children[par]) {
      const Box &ob = h->footprint[o];
      bool overlap = true;
      for (int a = 0; a < 3; ++a) overlap = overlap && b.lo[a] < ob.hi[a] && ob.lo[a] < b.hi[a];
      if (overlap) return bail(fail(PPM_EINVAL, "patches %d and %d overlap", o, p));
      if (place[o].refine != r)
        return bail(fail(PPM_EINVAL, "children of patch %d differ in refinement factor", par));
    }
    h->children[par].push_back(p);
  }
  const ppm_patch &root = patches[h->members[0][0]];
  if (root_kinds) {
    h->root_periodic = false;
    std::memcpy(h->root_kinds, root_kinds, sizeof h->root_kinds);
    if (root_inflow) {
      h->has_inflow = true;
      std::memcpy(h->root_inflow, root_inflow, sizeof h->root_inflow);
    }
  } else if (root.bc != PPM_BC_PERIODIC) {
    return bail(fail(PPM_EINVAL, "a root without boundary kinds must be PPM_BC_PERIODIC"));
  }
  ppm_status st = ppm_plan_create(&h->all, patches, npatch, nlevels, prec, params, "persistent=0",
                                  hip_stream);
  if (st != PPM_OK) return bail(st);
  if ((st = ppm_set_hierarchy(h->all, place, hip_stream)) != PPM_OK) return bail(st);
  h->lplan.assign(size_t(nlevels), nullptr);
  for (int l = 0; l < nlevels; ++l) {
    if (h->members[l].empty()) continue;
    std::vector<ppm_patch> lp;
    for (int32_t p : h->members[l]) lp.push_back(patches[p]);
    // per-sweep launches over all of a level's patches (faster than a
    // workgroup per patch for many small patches)
    if ((st = ppm_plan_create(&h->lplan[l], lp.data(), int32_t(lp.size()), nlevels, prec, params,
                              "persistent=0", hip_stream)) != PPM_OK)
      return bail(st);
  }
  hipError_t e;
  if ((e = hipMalloc(&h->d_dt, sizeof(double) * size_t(nlevels))) != hipSuccess ||
      (e = hipMalloc(&h->d_cfl, sizeof(double) * size_t(nlevels))) != hipSuccess)
    return bail(hip_fail(e, "timestep arrays"));
  if ((st = build_lists(h)) != PPM_OK) return bail(st);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return bail(hip_fail(e, "set-up"));
  h->t.assign(size_t(nlevels), 0.0);
  h->t_old.assign(size_t(nlevels), 0.0);
  h->nsteps.assign(size_t(nlevels), 0);
  h->stepped.assign(size_t(nlevels), 0);
  *out = h;
  return PPM_OK;
}

ppm_status ppm_amr_destroy(ppm_amr *h) {
  destroy(h);
  return PPM_OK;
}

ppm_status ppm_amr_step(ppm_amr *h, void *hip_stream) {
  if (!h) return fail(PPM_EINVAL, "hierarchy is NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  h->log.clear();
  ppm_status st = evolve(h, 0, 0.0, false, s);
  if (st != PPM_OK) return st;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "W-cycle");
  return PPM_OK;
}

ppm_status ppm_amr_set_expansion(ppm_amr *h, const double *a_dev) {
  if (!h) return fail(PPM_EINVAL, "hierarchy is NULL");
  for (ppm_plan *p : h->lplan)
    if (p) ppm_set_expansion(p, a_dev);
  h->expand = a_dev;
  return PPM_OK;
}

ppm_status ppm_amr_times(ppm_amr *h, double *t, int64_t *steps) {
  if (!h) return fail(PPM_EINVAL, "hierarchy is NULL");
  for (int l = 0; l < h->nlevels; ++l) {
    if (t) t[l] = h->t[l];
    if (steps) steps[l] = h->nsteps[l];
  }
  return PPM_OK;
}

ppm_status ppm_amr_step_log(ppm_amr *h, int32_t *levels, double *dts, int32_t capacity,
                            int32_t *count) {
  if (!h || !count) return fail(PPM_EINVAL, "hierarchy or count is NULL");
  *count = int32_t(h->log.size());
  for (int32_t i = 0; i < *count && i < capacity; ++i) {
    if (levels) levels[i] = h->log[size_t(i)].first;
    if (dts) dts[i] = h->log[size_t(i)].second;
  }
  return PPM_OK;
}

ppm_status ppm_amr_event_counts(ppm_amr *h, int64_t *fallback_faces, int64_t *floored_cells,
                                void *hip_stream) {
  if (!h) return fail(PPM_EINVAL, "hierarchy is NULL");
  int64_t fb = 0, fl = 0;
  for (ppm_plan *p : h->lplan) {
    if (!p) continue;
    int64_t a = 0, b = 0;
    ppm_status st = ppm_event_counts(p, &a, &b, 0, hip_stream);
    if (st != PPM_OK) return st;
    fb += a;
    fl += b;
  }
  if (fallback_faces) *fallback_faces = fb;
  if (floored_cells) *floored_cells = fl;
  return PPM_OK;
}

}  // extern "C"
