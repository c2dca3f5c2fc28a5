/*
 * ppm_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the dimensionally split
 * direct-Eulerian PPM update of the Enzo method paper (arXiv:1307.2265,
 * Sec. "Hydrodynamics: The PPM method", Eqs. mass_diff, momentum_diff,
 * energy_diff, gasenergy_diff, the dual-energy selection rules, the
 * two-shock Riemann solver with HLL fallback of Sec. "Riemann Solvers and
 * Fallback", and the hydro CFL condition of Sec. "Timestepping").  The
 * reconstruction, steepening, flattening and characteristic tracing that the
 * paper defers to Colella & Woodward (1984, "CW84") follow CW84's equations
 * 1.6-1.10, 1.14-1.17, 3.5-3.7 and its appendix, as read for a uniform grid.
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may call
 * this library.  It shares no code with the HIP path.
 *
 * What pins it (tests/test_oracle_*.py): the exact Riemann solution (Sod star
 * state, jump conditions, shock-shock problems where two-shock is exact), exact
 * translation of a quadratic profile and the flux it carries (reconstruction
 * and domain averages), second-order convergence of smooth and acoustic waves,
 * Sod E1 convergence, no new extrema, conservation, uniform state, mirror
 * symmetry, 1-D embedded in 3-D, flux-register identity, the CFL definition,
 * the steepening and flattening thresholds, the dual-energy selection rules
 * (eta1 cold flow, eta2 neighbourhood maximum), the flux of a flattened shock
 * face, and the HLL fallback on a vacuum-forming rarefaction.  The HLL flux
 * inside the wave fan equals the flux the exact solution's average over the
 * fan implies (integral conservation over the space-time box of the outer
 * wave speeds), face velocity included; a cell still non-positive after the
 * fallback is floored with its old velocity (density floor) or keeps the
 * momentum of its update (pressure floor), at the floor pressure.  The HLLC
 * solver (flag PPMO_HLLC, in place of two-shock) is pinned by the
 * Rankine-Hugoniot conditions across its outer waves and contact, exact
 * isolated contacts (stationary and moving), consistency, supersonic
 * upwinding, mirror symmetry, second-order agreement with the exact solution
 * for weak waves and with two-shock on smooth flow, Sod E1 convergence, a
 * stationary contact held to round-off and conservation.  The domain
 * boundary fill (ppmo_fill_boundary) is pinned by: periodic faces equal to
 * the periodic fill; reflecting walls evolving bit for bit as half of the
 * mirrored periodic box of twice the size; Sod between outflow faces against
 * the exact solution; uniform inflow-to-outflow flow staying uniform.  The
 * SecondOrderA parent interpolation is pinned by the paper's own 1-D and 2-D
 * formulas (data varying along one or two axes), exact linear fields,
 * conservation of the coarse value, and every corner of the interpolant
 * lying between the cell value and that corner's parent average; the patch
 * fill from the parent on linear conserved fields, and the sibling copy on a
 * tiling of one region by two patches.
 *
 * Parity unpinned (pinned only by these readings and by GPU == oracle):
 *   - the CW84 flattening slope omega_2 = 10 (f~ rises from 0 at a pressure
 *     ratio of omega_1 = 0.75 to 1 at 0.85; only the end points are pinned);
 *   - the HLL fallback's choice of the Davis wave-speed estimates (the pin
 *     of its flux takes them as given);
 *   - the Newton tolerance and iteration cap of the two-shock solver;
 *   - HLLC's outer wave speeds (the Davis estimates of the HLL fallback; the
 *     paper names none) and the internal energy carried with the density
 *     across its star states;
 *   - the diffusive flux (flag PPMO_DIFFUSION): its coefficient K = 0.1
 *     and its form along the sweep (CW84's multidimensional divergence is
 *     not used); pinned only by properties: nothing changes where the flow
 *     does not converge, conservation, fewer post-shock oscillations;
 *   - SecondOrderA's readings: corner values as 8-cell averages, the printed
 *     sign of the adjustment factor (read so the slopes sum to dQ0 s'), no
 *     epsilon (the selected slopes never sum to zero), the dQ0 = 0 case, and
 *     the interpolation of rho, rho v, rho E, rho e.
 *
 * Conventions (all host pointers, owned by the caller):
 *   - A grid has nx*ny*nz active cells and `ghost` ghost layers per side (3, as
 *     the paper's PPM stencil needs; 3..6 accepted).  With 3 layers the CW84
 *     flattening coefficient of the outermost reconstructed cell cannot see its
 *     outer neighbour and omits it; 4 layers give every needed cell its full
 *     stencil.
 *     Every field is an array of (nz+2g)*(ny+2g)*(nx+2g) doubles, x fastest.
 *   - Fields: rho (density), vx, vy, vz (velocity), etot (specific total
 *     energy E), eint (specific internal energy e, the dual-energy field).
 *   - flux_reg (nullable) receives dt*F at the six active-region boundary
 *     faces: [face: -x,+x,-y,+y,-z,+z][field: rho,mx,my,mz,E,e][t2][t1],
 *     t1/t2 the two transverse axes in increasing order (t1 fastest); faces
 *     normal to x hold ny*nz values per field, y: nx*nz, z: nx*ny.
 * Return values: 0 on success, -1 on an invalid argument.
 */
#ifndef PPM_ORACLE_H
#define PPM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PPMO_STEEPEN = 1u,      /* CW84 contact steepening of the density parabola */
  PPMO_FLATTEN = 2u,      /* CW84 appendix shock flattening */
  PPMO_DUAL_ENERGY = 4u,  /* eta1 pressure selection and eta2 resync */
  PPMO_FALLBACK_HLL = 8u, /* re-solve faces of non-positive cells with HLL */
  PPMO_HLLC = 16u,        /* HLLC face fluxes instead of the two-shock solver */
  PPMO_DIFFUSION = 32u    /* CW84's diffusive flux where the flow converges */
};

typedef struct {
  double gamma;        /* ratio of specific heats, > 1 */
  double cfl;          /* kappa_hydro in (0, 1] */
  double eta1, eta2;   /* dual-energy thresholds (1e-3 and 0.1 in the paper) */
  double rho_floor, p_floor, e_floor;
  double riemann_rtol; /* relative convergence tolerance on p* */
  int32_t riemann_max_iter;
  uint32_t flags;
  double a, adot;      /* expansion factor and its rate at the half step (1, 0: static) */
} ppmo_params;

typedef struct {
  int32_t nx, ny, nz, ghost;
  double dx, dy, dz;
  double *rho, *vx, *vy, *vz, *etot, *eint;
  double *flux_reg; /* nullable */
  double *gx, *gy, *gz; /* nullable: gravitational acceleration at the cell centres at the
                           half step (all three or none), same layout as the fields */
} ppmo_grid;

/* Counters of the rare numerical events of a sweep or step. */
typedef struct {
  int64_t fallback_faces; /* faces re-solved with HLL */
  int64_t floored_cells;  /* cells still non-positive after the fallback */
} ppmo_counts;

/* Number of doubles one grid's flux register holds. */
int64_t ppmo_flux_reg_size(int32_t nx, int32_t ny, int32_t nz);

/* One full step: three 1-D sweeps in the order given by sweep_order
 * (0:xyz 1:zyx 2:xzy 3:yxz 4:yzx 5:zxy).  Sweep k updates the cells that are
 * active along the axes already swept and along its own axis, and every
 * index (ghosts included) along the axes still to come.  counts may be NULL. */
int ppmo_step(ppmo_grid *g, const ppmo_params *p, double dt, int32_t sweep_order,
              ppmo_counts *counts);

/* One sweep along `axis` (0,1,2).  Bit a of active_mask set means the
 * transverse axis a is restricted to its active range, else all indices. */
int ppmo_sweep(ppmo_grid *g, const ppmo_params *p, double dt, int32_t axis,
               int32_t active_mask, ppmo_counts *counts);

/* One 1-D pencil of n = N + 2*ghost cells, updated in place (active cells
 * ghost..n-ghost-1).  u is the normal velocity, v1/v2 the transverse ones.
 * reg_lo/reg_hi (nullable) receive dt*(F_rho, F_u, F_v1, F_v2, F_E, F_e) at the
 * first and last active faces. */
int ppmo_pencil(const ppmo_params *p, int32_t n, int32_t ghost, double dt, double dx,
                double *rho, double *u, double *v1, double *v2, double *etot,
                double *eint, double *reg_lo, double *reg_hi, ppmo_counts *counts);

/* Expansion terms of the comoving equations (Sec. "Physical Equations", split
 * from the sweeps and solved implicitly and time-centred over dt with H =
 * adot / a of the parameters): peculiar velocity x (1 - H dt/2)/(1 + H dt/2),
 * specific total energy x (1 - H dt)/(1 + H dt), specific internal energy
 * x (1 - 3(gamma-1) H dt/2)/(1 + 3(gamma-1) H dt/2), over the active cells. */
int ppmo_expansion(ppmo_grid *g, const ppmo_params *p, double dt);

/* max over active cells of sum_d (c_s + |v_d|)/dx_d, and kappa a / that max. */
double ppmo_cfl_signal_max(const ppmo_grid *g, const ppmo_params *p);
double ppmo_cfl_dt(const ppmo_grid *g, const ppmo_params *p);

/* Periodic ghost fill of all six fields: q(ghost i) = q(active image of i). */
int ppmo_fill_periodic(ppmo_grid *g);

/* Domain boundary conditions of a grid face (Sec. "Boundary conditions"). */
enum {
  PPMO_FACE_PERIODIC = 0,   /* the image across the domain */
  PPMO_FACE_REFLECTING = 1, /* mirror image, normal velocity reversed */
  PPMO_FACE_OUTFLOW = 2,    /* copy of the edge cell */
  PPMO_FACE_INFLOW = 3      /* fixed values */
};

/* Ghost fill by per-face boundary conditions, faces -x,+x,-y,+y,-z,+z.
 * Axes are filled in order x, y, z; axis a covers its ghost layers, the axes
 * filled before it over their whole extent and the later axes over their
 * active range, so edges and corners compose the faces' rules.  inflow
 * (nullable unless a face is INFLOW): [face][rho, vx, vy, vz, etot, eint].
 * Periodic faces come in pairs; a reflecting axis needs at least `ghost`
 * active cells.  Returns -1 on an invalid argument. */
int ppmo_fill_boundary(ppmo_grid *g, const int32_t kinds[6], const double *inflow);

/* SecondOrderA interpolation (Appendix "Interpolation") of the centre of a
 * 3x3x3 coarse neighbourhood nb27[dz][dy][dx] to its r^3 fine cells
 * out[k][j][i]. */
void ppmo_second_order_a(const double *nb27, int32_t r, double *out);

/* Ghost cells of fine grid `fine` (its first active cell at global index
 * fine_start of its level) by SecondOrderA interpolation of the conserved
 * quantities of its parent grid (first active cell at parent_start of the
 * coarser level, refinement factor r >= 2).  -1 if a needed coarse cell or
 * one of its neighbours lies outside the parent array. */
int ppmo_fill_from_parent(ppmo_grid *fine, const int32_t fine_start[3], const ppmo_grid *parent,
                          const int32_t parent_start[3], int32_t r);

/* Ghost cells of dst that lie in the active region of src (same level) take
 * src's values. */
int ppmo_copy_from_sibling(ppmo_grid *dst, const int32_t dst_start[3], const ppmo_grid *src,
                           const int32_t src_start[3]);

/* A box of active cells [lo, hi) of a grid, in active-local indices (the
 * footprint of a finer patch, in this grid's cells). */
typedef struct {
  int32_t lo[3], hi[3];
} ppmo_box;

/* ppmo_step that also records, for every box, dt * F through its six faces
 * (faces lo[a]-1/2 and hi[a]-1/2 of each axis a, during the sweep along a)
 * into out: per box, in order, a block laid out like the flux register of a
 * grid with the box's dimensions.  Boxes lie inside the active region. */
int ppmo_step_capture(ppmo_grid *g, const ppmo_params *p, double dt, int32_t order,
                      ppmo_counts *counts, const ppmo_box *boxes, int32_t nboxes, double *out);

/* Flux correction (Sec. "Flux correction") of coarse grid C after its
 * children -- the finer patches whose footprints are boxes[0..nboxes), each
 * at least one cell inside C's active region, refinement factor r -- have
 * reached C's time.  caps: the coarse fluxes recorded by ppmo_step_capture
 * for the same boxes; fine_sums: per box, the child's flux register summed
 * over its substeps (its layout, dimensions r times the box's).  Every coarse
 * cell that shares a face with a box and lies in no box has the conserved
 * quantities rho, rho v, rho E and rho e corrected by the difference between
 * the coarse flux and the area average of the r^2 fine fluxes through that
 * face, divided by a dx; contributions are summed per cell in box, face
 * order and applied once. */
int ppmo_flux_correct(ppmo_grid *C, const ppmo_params *p, const ppmo_box *boxes,
                      int32_t nboxes, const double *caps, const double *fine_sums, int32_t r);

/* Projection (Sec. "Projection"): every coarse cell of `box` (inside C's
 * active region) gets the volume average of the conserved quantities rho,
 * rho v, rho E, rho e of the r^3 cells of fine grid F that cover it (F's
 * active region is exactly the box refined by r); v, E and e are stored as
 * the averages' ratios to the averaged density. */
int ppmo_project(ppmo_grid *C, const ppmo_box *box, const ppmo_grid *F, int32_t r);

/* Two-shock Riemann solver on (rho,u,p) left/right states.
 * out[0]=p*, out[1]=u*, out[2..4] = sampled (rho,u,p) at x/t=0,
 * out[5] = iterations taken, out[6] = 1 if the left side is upwind. */
void ppmo_two_shock(const ppmo_params *p, const double left[3], const double right[3],
                    double out[7]);

/* HLL flux (Davis wave speeds) on traced states (rho,u,v1,v2,p), each
 * state's internal energy being p/((gamma-1) rho):
 * out = F_rho, F_u, F_v1, F_v2, F_E, F_e, face velocity. */
void ppmo_hll_flux(const ppmo_params *p, const double left[5], const double right[5],
                   double out[7]);

/* HLLC flux (Davis outer wave speeds, contact speed from the Rankine-Hugoniot
 * conditions of the outer waves) on the same traced states and with the same
 * output layout as ppmo_hll_flux; out[6] is the contact speed S* inside the
 * wave fan, else the upwind normal velocity. */
void ppmo_hllc_flux(const ppmo_params *p, const double left[5], const double right[5],
                    double out[7]);

/* Exact Riemann solution of the Euler equations (ideal gas) by bisection on
 * the pressure function; samples rho,u,p at x/t = xi[k].  star[0]=p*,
 * star[1]=u*, star[2]=rho*_L, star[3]=rho*_R. */
void ppmo_exact_riemann(double gamma, const double left[3], const double right[3],
                        int32_t nxi, const double *xi, double *rho, double *u,
                        double *p, double star[4]);

/* Algorithmic operation counts of one step on the given grid (the grid is
 * advanced exactly as ppmo_step does).  ops = {add/sub, mul, div, sqrt,
 * compare, cell-sweeps performed}. */
int ppmo_count_ops(ppmo_grid *g, const ppmo_params *p, double dt, int32_t sweep_order,
                   int64_t ops[6]);

/* Threads the OpenMP runtime will use (1 without OpenMP). */
int ppmo_num_threads(void);
/* Host threads of the following calls (OpenMP over independent pencils;
   the results do not depend on it).  n < 1 is ignored. */
void ppmo_set_num_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
