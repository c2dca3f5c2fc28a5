/*
 * ppm.h -- C ABI of the MI355X PPM hydrodynamics library (libppm.so).
 *
 * The library advances block-structured grid patches by one step of the
 * dimensionally split, direct-Eulerian piecewise parabolic method described
 * in the Enzo method paper (arXiv:1307.2265), Sec. "Hydrodynamics: The PPM
 * method": per 1-D sweep, dual-energy pressure (Sec. "The dual energy
 * formulation", pressure selection rule with eta1), CW84 parabolic
 * reconstruction with monotonicity limiting, contact steepening and shock
 * flattening, characteristic tracing, a two-shock Riemann solver with HLL
 * fallback (Sec. "Riemann Solvers and Fallback"), the conservative update
 * (Eqs. mass_diff, momentum_diff, energy_diff) with the internal-energy
 * update (Eq. gasenergy_diff) and the eta2 resync (Eq. dualselect), the
 * boundary fluxes that flux correction needs (Sec. "Flux correction"), and
 * the hydro CFL timestep (Sec. "Timestepping", harmonic multi-D form).
 * Optionally, the gravity source terms of Eqs. momentum_diff and energy_diff
 * from a caller-supplied acceleration field (ppm_patch gx, gy, gz) and the
 * comoving-coordinate terms of Sec. "Physical Equations" from per-level
 * expansion factors (ppm_set_expansion, ppm_expansion); without them the
 * static equations (a = 1, g = 0) are solved.
 *
 * Data layout.  Every patch holds nx*ny*nz active cells surrounded by `ghost`
 * ghost layers (Sec. "Adaptive mesh refinement": 3 for PPM).  Each field is a
 * separate device array of (nz+2g)*(ny+2g)*(nx+2g) elements, x fastest.
 * Fields: rho (density), vx, vy, vz (velocity), etot (specific total energy
 * E = e + |v|^2/2), eint (specific internal energy e, the dual-energy field).
 * PPM_FP64 stores all six as double and computes in double.  PPM_MIXED
 * stores rho, vx, vy, vz as float and etot, eint as double.  It reconstructs,
 * traces, samples the Riemann solution and forms the mass, momentum and
 * internal-energy fluxes and the rho and v updates in float; it keeps the
 * two-shock Newton iteration for p*, the total-energy flux, the total and
 * internal energy accumulation (and their division by the new density), the
 * dual-energy selection (eta1, eta2), the HLL fallback, the flux registers
 * and the CFL timestep in double.
 *
 * Flux registers (optional, per patch, device, double): dt * F at the six
 * faces of the active region, laid out
 *   [face: -x,+x,-y,+y,-z,+z][field: rho, mx, my, mz, E, e][t2][t1]
 * with t1 < t2 the axes transverse to the face (t1 fastest), so a face normal
 * to x holds ny*nz values per field, normal to y nx*nz, normal to z nx*ny.
 * The mass flux through a face is rho*u, the momentum fluxes rho*u*v (+p on
 * the normal component), the energy flux rho*u*E + u*p, and the internal
 * energy flux rho*u*e; the p div v term of the internal-energy equation is a
 * source, not a flux, and is not recorded.
 *
 * Ownership.  The caller owns every field, register and dt array (device
 * memory, e.g. torch tensors); a plan owns only its own metadata and
 * workspace.  ppm_fill_periodic, ppm_cfl_dt, ppm_step and ppm_sweep allocate
 * nothing and only enqueue work on the given stream, so they can be captured
 * into a HIP graph; dt stays on the device between them.  A plan must be
 * used from one stream at a time.
 *
 * Errors.  Every call validates its arguments before it launches anything
 * and returns PPM_EINVAL (nothing launched) with a message readable through
 * ppm_last_error() (thread-local).  HIP runtime failures return PPM_EHIP.
 * Numerical events (HLL fallback faces, floored cells) are counters, not
 * errors.
 */
#ifndef PPM_H
#define PPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PPM_OK = 0,
  PPM_EINVAL = -1,      /* invalid argument; nothing was launched */
  PPM_ENOMEM = -2,      /* device or host allocation failed (plan creation only) */
  PPM_EHIP = -3,        /* a HIP runtime call failed */
  PPM_EUNSUPPORTED = -4 /* a valid request the library does not support */
} ppm_status;

typedef enum { PPM_FP64 = 0, PPM_MIXED = 1 } ppm_precision;

/* Where a patch's ghost values come from. */
enum {
  PPM_BC_PERIODIC = 0, /* ppm_fill_periodic fills them from the patch's own active cells */
  PPM_BC_SUPPLIED = 1  /* the caller fills them (e.g. from a parent or sibling grid);
                          ppm_fill_periodic leaves the patch untouched */
};

enum {
  PPM_STEEPEN = 1u,      /* contact steepening of the density parabola */
  PPM_FLATTEN = 2u,      /* shock flattening of all parabolas */
  PPM_DUAL_ENERGY = 4u,  /* eta1 pressure selection and eta2 resync of e */
  PPM_FALLBACK_HLL = 8u, /* re-solve the faces of non-positive cells with HLL */
  PPM_ALL_FLAGS = 15u,   /* the four above: the paper's PPM with two-shock */
  PPM_HLLC = 16u,        /* face fluxes by the HLLC solver (Sec. "Riemann Solvers
                            and Fallback"; Davis outer wave speeds, contact speed
                            from the outer waves' jump conditions) instead of
                            two-shock; the HLL fallback still applies */
  PPM_DIFFUSION = 32u    /* the optional diffusive flux (Sec. "Hydrodynamics: The
                            PPM method", after CW84): where the flow converges
                            across a face (u_l > u_r of the sweep input), every
                            conserved quantity's flux gains 0.1 (u_l - u_r)(Q_l -
                            Q_r); on the Riemann and on the HLL fallback flux */
};

/* One grid patch.  All pointers are device pointers owned by the caller. */
typedef struct {
  int32_t nx, ny, nz; /* active cells per axis, >= 1 */
  int32_t ghost;      /* ghost layers per side, 3..6 (3 in the paper) */
  int32_t level;      /* index into the per-level dt array, 0 <= level < nlevels */
  int32_t bc;         /* PPM_BC_PERIODIC or PPM_BC_SUPPLIED */
  double dx, dy, dz;  /* cell widths, > 0 */
  void *rho, *vx, *vy, *vz; /* double (PPM_FP64) or float (PPM_MIXED) */
  double *etot, *eint;      /* double in both precisions.  Every cell a sweep
                               reads, ghosts included, must hold a physical
                               state: finite values, rho >= rho_floor, and
                               magnitudes below 1e100 (results for other
                               input are unspecified; none is detected) */
  double *flux_reg;         /* nullable; ppm_flux_reg_size(nx,ny,nz) doubles */
  const void *gx, *gy, *gz; /* nullable (all three or none): gravitational
                               acceleration at the cell centres at the half
                               step, in rho's type and layout, over the whole
                               ghosted box (the sweeps also update ghost cells);
                               read by every sweep, whose update then adds the
                               source terms of Eqs. momentum_diff and
                               energy_diff.  Zero-initialise for no gravity. */
} ppm_patch;

typedef struct {
  double gamma;            /* ratio of specific heats, > 1 */
  double cfl;              /* kappa_hydro, 0 < cfl <= 1 */
  double eta1, eta2;       /* dual-energy thresholds (paper: 1e-3, 0.1) */
  double rho_floor, p_floor, e_floor; /* floors (Sec. "Riemann Solvers and Fallback": a
                                          cell still non-positive after the HLL re-solve is
                                          raised to them): rho_floor, p_floor >= 1e-100
                                          (they bound the operands of the fast FP64
                                          division and square root), e_floor > 0.
                                          PPM_MIXED stores the density in float, so its
                                          rho_floor and p_floor must also be normal floats
                                          (>= FLT_MIN = 1.1754944e-38, <= FLT_MAX), and the
                                          plan raises each to the nearest float at or above
                                          it, the floor that a stored density can hold
                                          exactly.  PPM_EINVAL otherwise */
  double riemann_rtol;     /* relative tolerance on the two-shock p*, > 0 */
  int32_t riemann_max_iter;/* Newton iteration cap, >= 1 */
  uint32_t flags;          /* PPM_STEEPEN | PPM_FLATTEN | ... */
} ppm_params;

typedef struct ppm_plan ppm_plan;

/* Number of doubles in one patch's flux register. */
int64_t ppm_flux_reg_size(int32_t nx, int32_t ny, int32_t nz);

/* Create a plan over `npatch` patches (host array, copied): each patch is an
 * independent problem with Dirichlet ghost data and every patch of a level
 * shares that level's timestep (Secs. "Adaptive Mesh Refinement" and
 * "Timestepping").  nlevels is the
 * length of every dt array later passed in.  tile_config (nullable) is a
 * text of "key=value" pairs separated by spaces that overrides the launch
 * shapes; unknown keys are an error.  Keys:
 *   lanes=M        axis bitmask: sweeps along axis a (bit a) give each pencil
 *                  to a wavefront with its cells across the lanes (pencils of
 *                  at most 64 cells are packed side by side, 64/n per wave);
 *                  the other sweeps give each pencil to one thread that
 *                  marches it.  Default 1 (x only), except for one patch
 *                  with (nx + 2 ghost)(nz + 2 ghost) below 128 x the number
 *                  of compute units (too few pencils to fill the device one
 *                  thread each) and a tile_config that sets none of lanes,
 *                  block, tail and tail_round: then 7 (every axis).
 *   block=B        threads per block of the marching kernel (64..256;
 *                  default 256 for one patch, 64 for several).
 *   lanes_block=B  threads per block of the lane-parallel kernel (64..256;
 *                  default 256 for one patch, 64 for several).
 *   cfl_cells=C    active cells per block of the CFL reduction.
 *   group=0|1      marching sweeps number the pencils of patches of equal
 *                  pencil length consecutively, so a wavefront may span
 *                  patches and none is left partly empty at a patch's end
 *                  (default 1 for several patches, 0 for one).
 *   persistent=0|1 ppm_step as one persistent launch: workgroups take whole
 *                  patches from a queue (largest first) and run their three
 *                  sweeps back to back; with 0, one launch per sweep over all
 *                  patches.  A workgroup owns a whole patch, so persistent=1
 *                  needs every patch to hold at most 2^21 active cells
 *                  (PPM_EINVAL otherwise).  Default: 1 for several patches
 *                  that all satisfy this, else 0.
 *   batch_block=B  threads per workgroup of the persistent launch (64..256).
 *   batch_blocks=W workgroups of the persistent launch (default: 512/B per CU).
 *   tail=0|1       one ungrouped patch: when a marching sweep's pencils
 *                  exceed a whole number of rounds of one marching block per
 *                  compute unit by at most an eighth of a round, march the
 *                  whole rounds and stream the rest with the lane-parallel
 *                  kernel, one pencil per wavefront, in a second launch
 *                  (default 1).
 *   tail_round=R   take R pencils (a multiple of block) as the round and give
 *                  any rest to the lane-parallel launch (for tests and tuning).
 *   split=0|1      one ungrouped patch: a marching sweep with fewer pencils
 *                  than two blocks per compute unit, of at least 16 active
 *                  cells each, runs two threads per pencil (each marches half
 *                  of it, from max(5, ghost) cells before its first own
 *                  cell), which
 *                  doubles the waves on a device the pencils cannot fill
 *                  (default 1).
 * Results do not depend on the launch shapes.  Uploads the patch table to
 * the device on `hip_stream` (0 = default stream) and allocates the event
 * counters.  On success *out owns the plan. */
ppm_status ppm_plan_create(ppm_plan **out, const ppm_patch *patches, int32_t npatch,
                           int32_t nlevels, ppm_precision prec, const ppm_params *params,
                           const char *tile_config, void *hip_stream);

/* Release a plan (synchronises with nothing; the caller must make sure no
 * enqueued work still uses it).  NULL is accepted. */
ppm_status ppm_plan_destroy(ppm_plan *plan);

/* Periodic ghost fill (Sec. "Boundary conditions", the periodic kind) of
 * every PPM_BC_PERIODIC patch of the plan (each is
 * treated as a periodic box of its own): ghost cell i takes the value of the
 * active cell g + ((i - g) mod N) along every axis.  PPM_BC_SUPPLIED patches
 * are not touched. */
ppm_status ppm_fill_periodic(ppm_plan *plan, void *hip_stream);

/* Domain boundary conditions of a face (Sec. "Boundary conditions"). */
typedef enum {
  PPM_FACE_PERIODIC = 0,   /* q(ghost) = q(the image across the patch) */
  PPM_FACE_REFLECTING = 1, /* mirror image about the face, normal velocity reversed */
  PPM_FACE_OUTFLOW = 2,    /* copy of the edge cell */
  PPM_FACE_INFLOW = 3      /* fixed values */
} ppm_face_kind;

/* Ghost fill of patch `patch` of the plan (any bc) by per-face domain
 * boundary conditions: kinds[6] (host) for the faces -x,+x,-y,+y,-z,+z;
 * inflow (host, nullable unless a face is PPM_FACE_INFLOW) holds
 * [face][rho, vx, vy, vz, etot, eint] (copied at the call; narrowed to the
 * field precision).  The result is that of filling the axes in order x, y,
 * z, each over the whole extent of the axes before it and the active range of
 * the axes after it, so edges and corners compose the faces' rules.
 * PPM_EINVAL (nothing launched) for a bad patch index or kind, a periodic
 * face whose opposite face is not periodic, a reflecting axis with fewer
 * active cells than ghost layers, or inflow faces without values. */
ppm_status ppm_fill_boundary(ppm_plan *plan, int32_t patch, const int32_t *kinds,
                             const double *inflow, void *hip_stream);

/* Place of a patch in the AMR hierarchy. */
typedef struct {
  int32_t parent;   /* index of the parent patch in the plan (level - 1), or -1 */
  int32_t refine;   /* refinement factor r >= 2 from the parent's cells to this patch's */
  int32_t start[3]; /* global index, in this patch's level, of its first active cell */
} ppm_patch_place;

/* Record the hierarchy of the plan's patches (host array of npatch, copied)
 * and build the device work lists of ppm_fill_ghosts: for every patch with a
 * parent, its ghost cells; for every pair of patches of one level, the ghost
 * cells of one that lie in the active region of the other.  PPM_EINVAL
 * (nothing changed) if a parent index is out of range or not one level
 * coarser, r < 2, or a ghost cell's parent cell or one of its 26 neighbours
 * lies outside the parent's array (ghosts included).  Allocates device
 * memory; call again to replace the hierarchy. */
ppm_status ppm_set_hierarchy(ppm_plan *plan, const ppm_patch_place *place, void *hip_stream);

/* Ghost cells of every patch of `level` that has a parent (Sec. "Boundary
 * conditions"): first SecondOrderA interpolation (Appendix "Interpolation")
 * of the parent's rho, rho v, rho E, rho e, stored as rho, v, E, e; then the
 * copy from every sibling of the level whose active region covers a ghost
 * cell.  The parents' ghosts must be valid (filled before, level by level).
 * Patches of the level without a parent are not touched.  PPM_EINVAL without
 * a recorded hierarchy. */
ppm_status ppm_fill_ghosts(ppm_plan *plan, int32_t level, void *hip_stream);

/* ---- AMR level step on a static hierarchy -------------------------------
 * The W-cycle of Sec. "Adaptive Mesh Refinement" (EvolveLevel) over a fixed
 * patch tree: the root takes one step with its CFL timestep; then every finer
 * level takes as many steps of its own CFL timestep as it needs to reach its
 * parent's time (the last one cut to land on it exactly), recursively; after
 * a level's children have caught up, the level's cells that share a face
 * with a child footprint are corrected with the difference between the
 * coarse flux through that face and the area average of the child's fluxes
 * summed over its substeps (Sec. "Flux correction"), and the cells a child
 * covers get the volume average of its conserved quantities (Sec.
 * "Projection").  Ghost zones are set at the start of a level's steps and
 * after each step: the root's by its domain boundary conditions, the others
 * by SecondOrderA interpolation from the parent's state at the patch's time
 * -- linear in time between the parent's states before and after its step --
 * and then from siblings (as ppm_fill_ghosts).
 *
 * patches / place: every patch and its placement as for ppm_set_hierarchy
 * (level from ppm_patch.level); exactly one root patch (level 0, parent -1);
 * every other patch needs a flux register, starts and ends on parent cell
 * boundaries, lies at least one parent cell inside its parent's active
 * region, does not overlap its siblings, and shares its refinement factor
 * with them.  root_kinds (nullable): the root's six domain boundary kinds as
 * for ppm_fill_boundary (with root_inflow); NULL means periodic, which needs
 * a PPM_BC_PERIODIC root.  The hierarchy keeps pointers to the caller's
 * fields and registers, allocates a copy of the fields of every patch that
 * has children (its state before its last step), and a few small device
 * work lists. */
typedef struct ppm_amr ppm_amr;
ppm_status ppm_amr_create(ppm_amr **out, const ppm_patch *patches, const ppm_patch_place *place,
                          int32_t npatch, int32_t nlevels, ppm_precision prec,
                          const ppm_params *params, const int32_t *root_kinds,
                          const double *root_inflow, void *hip_stream);
ppm_status ppm_amr_destroy(ppm_amr *amr); /* NULL is accepted */

/* One root step of the W-cycle.  The host reads each level's timestep from
 * the device before that level's step (one small copy and a stream
 * synchronisation per level step) and returns after the stream has finished. */
ppm_status ppm_amr_step(ppm_amr *amr, void *hip_stream);

/* Comoving coordinates for the whole hierarchy: a_dev as for
 * ppm_set_expansion (2 * nlevels doubles, a and adot of each level at its
 * half step, read by every launch; NULL: static).  Each level step then also
 * applies the split expansion terms (ppm_expansion) to its patches after its
 * sweeps, over the same dt. */
ppm_status ppm_amr_set_expansion(ppm_amr *amr, const double *a_dev);

/* Current time and steps taken of every level (arrays of nlevels, nullable). */
ppm_status ppm_amr_times(ppm_amr *amr, double *t, int64_t *steps);

/* The (level, dt) of every level step of the last ppm_amr_step, in the order
 * taken: *count gets their number, the first `capacity` are written. */
ppm_status ppm_amr_step_log(ppm_amr *amr, int32_t *levels, double *dts, int32_t capacity,
                            int32_t *count);

/* Event counters (HLL faces, floored cells) summed over the levels. */
ppm_status ppm_amr_event_counts(ppm_amr *amr, int64_t *fallback_faces, int64_t *floored_cells,
                                void *hip_stream);

/* Comoving coordinates (Sec. "Physical Equations").  a_dev: device array of
 * 2 * nlevels doubles, owned by the caller, holding for each level l the
 * expansion factor a_l = a_dev[2l] > 0 and its rate adot_l = a_dev[2l+1] at
 * the level's half step.  From this call on every sweep divides its flux
 * differences by a_l (time ratio dt / (a_l dx)) and its gravity source by
 * a_l, and the CFL timestep becomes cfl a_l / max; the values are read by each
 * launch, so the caller may change them between steps without a new plan.  A
 * graph made by ppm_graph_create keeps the pointer the plan had when it was
 * made.  NULL restores the static equations (a = 1).  Values that are not
 * positive and finite give meaningless results (no error is detected on the
 * device). */
ppm_status ppm_set_expansion(ppm_plan *plan, const double *a_dev);

/* The expansion terms of the comoving equations, split from the sweeps and
 * integrated over each level's dt (dt_dev[level]) implicitly and
 * time-centred with H = adot / a of the level: velocities times
 * (1 - H dt/2)/(1 + H dt/2), specific total energy times (1 - H dt)/(1 + H dt),
 * specific internal energy times (1 - x)/(1 + x), x = 3 (gamma - 1) H dt / 2;
 * active cells only.  Needs ppm_set_expansion (PPM_EINVAL otherwise). */
ppm_status ppm_expansion(ppm_plan *plan, const double *dt_dev, void *hip_stream);

/* Hydro CFL timestep per level (Sec. "Timestepping"):
 *   dt_dev[l] = cfl a_l / max over the active cells of the level's patches of
 *               sum_d (c_s + |v_d|) / dx_d,
 * with c_s from the same dual-energy pressure the sweeps use.  dt_dev is a
 * device array of nlevels doubles; levels without patches get +inf. */
ppm_status ppm_cfl_dt(ppm_plan *plan, double *dt_dev, void *hip_stream);

/* One full step of every patch with its level's dt (device array of nlevels
 * doubles): three 1-D PPM sweeps (Sec. "Hydrodynamics: The PPM method",
 * dimensionally split; Sec. "Solving the hydrodynamic equations on a grid"
 * for the one ghost fill per step) in the order sweep_order (0:xyz 1:zyx 2:xzy
 * 3:yxz 4:yzx 5:zxy).  The k-th sweep updates the cells that are active along
 * the axes swept so far and along its own axis, and every index (ghosts
 * included) along the axes still to come, so one ghost fill per step
 * suffices.  Fields are updated in place; flux registers (if given) are
 * overwritten with dt*F of the face's own sweep. */
ppm_status ppm_step(ppm_plan *plan, const double *dt_dev, int32_t sweep_order,
                    void *hip_stream);

/* One step as ppm_step with the per-level dt in dt_dev, after which dt_dev
 * holds the hydro CFL timestep of the new state -- the values ppm_cfl_dt
 * would return if called next, bit for bit.  The signal speeds are taken by
 * the step's last sweep from the values it stores, so no extra pass reads
 * the fields.  A loop calls ppm_cfl_dt once, then ppm_step_cfl every step
 * (ppm_fill_periodic before each, for periodic patches). */
ppm_status ppm_step_cfl(ppm_plan *plan, double *dt_dev, int32_t sweep_order, void *hip_stream);

/* One sweep along `axis` (0,1,2) of every patch; bit a of active_mask
 * restricts transverse axis a to its active range (else all indices). */
ppm_status ppm_sweep(ppm_plan *plan, const double *dt_dev, int32_t axis, int32_t active_mask,
                     void *hip_stream);

/* ppm_sweep that also folds the CFL signal speed of every cell it writes
 * into the plan's per-level maxima (the last sweep of a step, whose cells
 * are exactly the active ones); ppm_cfl_finalize then turns the maxima into
 * dt_dev[l] = cfl / max (+inf for a level without patches) and clears them.
 * ppm_cfl_dt is the same maxima over the current state followed by
 * ppm_cfl_finalize. */
ppm_status ppm_sweep_cfl(ppm_plan *plan, const double *dt_dev, int32_t axis,
                         int32_t active_mask, void *hip_stream);
ppm_status ppm_cfl_finalize(ppm_plan *plan, double *dt_dev, void *hip_stream);

/* Read (synchronising `hip_stream`) and optionally reset (reset != 0) the
 * plan's event counters of the positivity fallback (Sec. "Riemann Solvers and
 * Fallback"): faces re-solved with HLL, cells floored after the fallback. */
ppm_status ppm_event_counts(ppm_plan *plan, int64_t *fallback_faces, int64_t *floored_cells,
                            int32_t reset, void *hip_stream);

/* HIP graph of one step, for callers that launch the same step repeatedly
 * (and for capture-friendly batching): the parts selected by `parts`, in the
 * order fill -> CFL -> step (or step with the next dt), with the given dt
 * array and sweep order, are
 * captured once into an executable graph (on a private stream; nothing is
 * executed).  The graph records only kernel launches.  It refers to the
 * plan, its patches and dt_dev, which must outlive it. */
typedef struct ppm_graph ppm_graph;
enum { PPM_GRAPH_FILL = 1u, PPM_GRAPH_CFL = 2u, PPM_GRAPH_STEP = 4u,
       PPM_GRAPH_STEP_CFL = 8u /* ppm_step_cfl; excludes PPM_GRAPH_STEP */ };
ppm_status ppm_graph_create(ppm_graph **out, ppm_plan *plan, double *dt_dev,
                            int32_t sweep_order, uint32_t parts, void *hip_stream);
ppm_status ppm_graph_launch(ppm_graph *graph, void *hip_stream);
ppm_status ppm_graph_destroy(ppm_graph *graph); /* NULL is accepted */

/* The correctly rounded FP64 division and square root that the sweeps use
 * wherever their operands are bounded (the equation of state, the Riemann
 * solvers, the update), exposed so that a caller can check them against host
 * IEEE arithmetic: quot_dev[i] = a_dev[i] / b_dev[i] and root_dev[i] =
 * sqrt(a_dev[i]) for i < n, device arrays of n doubles (caller-owned), on
 * `hip_stream`.  Valid, i.e. equal to IEEE round-to-nearest, for finite
 * a, b with |a|, |b| and |a / b| in [1e-250, 1e250] and a > 0 for the root:
 * the range the floors (>= 1e-100) and state magnitudes (< 1e100) of
 * ppm_patch keep every operand in.  Outside it the results are unspecified
 * (no operand scaling, no special values).  PPM_EINVAL for n < 0 or NULL
 * arrays. */
ppm_status ppm_fp64_ops(const double *a_dev, const double *b_dev, double *quot_dev,
                        double *root_dev, int64_t n, void *hip_stream);

/* ---- A step that allocates nothing ---------------------------------------
 * For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ppm_step_cfl for up to PPM_NOALLOC_MAX_PATCHES patches without a plan.
 * The patch table, launch maps, event counters and per-level CFL maxima
 * live in a static device buffer of PPM_NOALLOC_SCRATCH_BYTES bytes that the
 * library holds on every device it runs on until the process ends (its
 * address is taken at the first call on that device); the call neither
 * allocates nor frees anything.  Every call on a device rewrites and reuses
 * that device's buffer: calls that overlap on one device (other host threads,
 * or other streams whose work is still running) race on it and must be
 * serialised by the caller.
 *
 * patches (host, npatch of them, 1..PPM_NOALLOC_MAX_PATCHES), nlevels
 * (1..PPM_NOALLOC_MAX_PATCHES), prec, params: as for ppm_plan_create
 * (default launch shapes).  dt_dev: device array of nlevels doubles.  parts:
 * PPM_NOALLOC_FILL first fills the ghosts of every patch periodically (all
 * patches must then be PPM_BC_PERIODIC), as ppm_fill_periodic;
 * PPM_NOALLOC_CFL then reduces dt_dev from the current state, as ppm_cfl_dt
 * (without it dt_dev holds the step's timesteps on entry).  Then one step in
 * sweep_order with dt_dev, after which dt_dev holds the CFL timestep of the
 * new state -- bit for bit what a plan over the same patches gives through
 * ppm_fill_periodic, ppm_cfl_dt and ppm_step_cfl.  events (host, nullable):
 * if given, the call waits for the stream and stores the step's HLL faces
 * and floored cells in events[0] and events[1].  PPM_EINVAL (nothing
 * launched) for more than PPM_NOALLOC_MAX_PATCHES patches or levels and for
 * every argument ppm_plan_create rejects. */
#define PPM_NOALLOC_MAX_PATCHES 16
#define PPM_NOALLOC_SCRATCH_BYTES 4096
enum { PPM_NOALLOC_FILL = 1u, PPM_NOALLOC_CFL = 2u };
ppm_status ppm_step_cfl_noalloc(const ppm_patch *patches, int32_t npatch, int32_t nlevels,
                                ppm_precision prec, const ppm_params *params, double *dt_dev,
                                int32_t sweep_order, uint32_t parts, int64_t *events,
                                void *hip_stream);

const char *ppm_status_str(ppm_status s);
const char *ppm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
