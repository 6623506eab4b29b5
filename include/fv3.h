/*
 * fv3.h -- C ABI of an MI355X-native implementation of the acoustic substep
 * loop of the FV3 finite-volume cubed-sphere dynamical core and of its tracer
 * transport.
 *
 * The paper (Sec. II) describes FV3 as three nested loops: the physics step,
 * the remapping step (which advects tracers and remaps the vertical), and the
 * innermost acoustic substep that integrates the nonhydrostatic dynamics on
 * Lagrangian surfaces, with halo exchanges at several points of each
 * substep.  It drives the whole time-stepping program as one call into a
 * compiled library (Fig. 2 caption, Sec. III-C).  This header exposes that
 * innermost loop and the tracer advection of the middle loop as such calls.
 *
 * Conventions shared by every entry point:
 *  - All pointers to field data are DEVICE pointers (HIP, one GPU) laid out
 *    as described by fv3_layout.  The caller allocates and frees them; the
 *    library never frees caller memory.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t passed as
 *    void*; NULL = the default stream).  Argument validation is synchronous:
 *    an invalid call returns an error and enqueues nothing.
 *  - Grids are created by fv3_init_grid, owned by the library, immutable after
 *    creation, and may be shared by concurrent calls on distinct states.
 *  - Errors found on the device (|Courant| > 1, non-finite prognostics) are
 *    latched per grid and returned by fv3_check_status.
 *  - fv3_last_error() returns a thread-local message for the last failure.
 */
#ifndef FV3_H
#define FV3_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FV3_OK = 0,
    FV3_EINVAL = -1,        /* bad argument value (NULL pointer, dt <= 0, n_split < 1, ...) */
    FV3_ESHAPE = -2,        /* sizes inconsistent with the grid or limits                   */
    FV3_EDTYPE = -3,        /* precision mode mismatch                                      */
    FV3_EDEVICE = -4,       /* HIP runtime error / no device                                */
    FV3_ENOMEM = -5,        /* device allocation failed (grid creation only)                */
    FV3_ECFL = -6,          /* a Courant number exceeded 1 in d_sw (latched on device)      */
    FV3_ENONFINITE = -7,    /* a prognostic became non-finite (latched on device)           */
    FV3_EUNSUPPORTED = -8,  /* option not implemented (a PPM order not listed below)        */
    FV3_EREMAP = -9,        /* reference interfaces not increasing in a column (latched)    */
    FV3_EINTERNAL = -99
} fv3_status;

typedef enum { FV3_GRID_DOUBLY_PERIODIC = 0, FV3_GRID_CUBED_SPHERE = 1 } fv3_grid_kind;
typedef enum { FV3_FP64 = 0, FV3_MIXED = 1 } fv3_precision;

/* Grid description.  Cubed sphere: 6 equiangular gnomonic tiles of n x n
 * cells (Sec. II), radius and rotation rate given.  Doubly periodic: one
 * n x n tile of spacing dx with constant Coriolis parameter f0.  Vertical:
 * nz Lagrangian layers below the model top pressure ptop.  hord selects the
 * PPM order of every horizontal transport (Lin-Rood fluxes of delp, pt, w,
 * vorticity and tracers, and the kinetic-energy faces): 8 the monotone order
 * (limited slopes, edge deviations clipped to twice the slope), 6 the
 * unlimited order (the same fourth-order edges and parabola without either
 * constraint), 5 the 2dx-filtered order (order 6, but the upwind cell mean
 * where that cell and a neighbour are both strict local extrema).  hord_tr,
 * if not 0, replaces hord in fv3_tracer_transport and also admits 7, the
 * positive-definite order (order 6 with each parabola of non-negative mean
 * scaled about its mean until its minimum over the cell is 0; non-negative
 * tracers stay non-negative).  Other values: FV3_EUNSUPPORTED.  pp_order
 * selects how both column solves carry the layer pressure perturbation to
 * the interfaces (Sec. IX-B): 2 (0 means the same) the mass-weighted mean of
 * the two adjacent layers, 4 the interface value of the cubic (in the mass
 * coordinate) whose means over the two layers on each side are theirs, with
 * the mass-weighted mean next to the top and the bottom; other values:
 * FV3_EUNSUPPORTED.  beta
 * in [0.5, 1] off-centres the semi-implicit vertical solve (Sec. IX-B): the
 * momentum equation sees beta P^{n+1} + (1 - beta) P* and the pressure
 * response is driven by beta w^{n+1} + (1 - beta) w^n; 1 is backward Euler
 * (outside [0.5, 1]: FV3_EINVAL).  d2_bg in [0, 0.25] turns
 * on del-2 divergence damping in d_sw: nu = d2_bg x (smallest dual-cell area
 * of the grid) times the divergence of the D-grid winds at each corner is
 * subtracted from the kinetic energy there, which diffuses the divergence
 * (outside [0, 0.25]: FV3_EINVAL).  dddmp in [0, 1] raises that coefficient
 * per corner to min(0.2, dddmp dt sqrt(DT^2 + DS^2)) where larger (the
 * Smagorinsky magnitude of the paper's Sec. VII-C case study; DT the tension
 * at the corner, DS the shear of its cells, dt the substep; it applies with
 * d2_bg = 0 too).  nord 1 or 2 with d4_bg in (0, 0.25] adds del-4 or del-6
 * damping: the corner divergence D of the D-grid winds gets nord corner
 * Laplacians (the same divergence operator applied to the gradient along
 * the cell edges, corner halo exchanged before each), and (-1)^(nord+1) nu
 * times the result is added to the kinetic energy, nu = (d4_bg x smallest
 * dual-cell area)^(nord+1), so that dD/dt = (-1)^nord nu Lap^(nord+1) D
 * (nord outside [0, 2]: FV3_EUNSUPPORTED; d4_bg outside [0, 0.25]:
 * FV3_EINVAL).  vtdm in (0, 0.25] adds del-2 vorticity damping: the
 * diffusive flux nu_v (w(upwind side) - w(cell)) x face length / centre
 * distance of the relative vorticity w joins the vorticity fluxes of the
 * momentum update, nu_v = vtdm x smallest dual-cell area (outside
 * [0, 0.25]: FV3_EINVAL).  edge_fix = 1 on the cube: a face on a tile edge
 * is stored by both tiles; after each flux-form transport (delp, pt delp,
 * w delp in d_sw, each tracer sub-cycle) both copies of its flux take their
 * mean and the cell next to the face takes the difference, so the global
 * sums of mass, pt mass and tracer masses are exact; the accumulated mass
 * fluxes take the mean too (no effect on the doubly periodic grid; other
 * values: FV3_EINVAL).  edge_ppm = 1 on the cube: every flux-form transport
 * (fv_tp_2d of delp, pt, w, the vorticity, the dz_d heights and the
 * tracers) builds the PPM edge values at the three interfaces around each
 * tile edge from one side only, the edge value itself as the mean of the two
 * width-weighted linear extrapolations to the edge (the panel-edge treatment
 * of Putman & Lin 2007); order 8 constrains the two cells beside the edge
 * and the second cell inside the tile to monotone parabolas (Colella &
 * Woodward 1984) instead of clipping to twice the slope.  Sweeps through the
 * corner halo keep the centred stencil.  No effect on the doubly periodic
 * grid; other values: FV3_EINVAL.  edge_interp = 1 on the cube (the edge
 * corrections of Sec. V-B): c_sw's D-grid to cell-centre and cell-centre to
 * C-grid interpolations and nh_p_grad's cell-to-corner interpolation, where
 * their four-point stencils would reach across a tile edge, use the
 * quadratic through the three nearest points on their own side (weights
 * 3/8, 3/4, -1/8 for the point values of c_sw, 1/3, 5/6, -1/6 for the cell
 * means of nh_p_grad), and a face or corner on the edge takes the mean of
 * the two linear extrapolations from the two nearest points of each side;
 * sweeps outside the tile keep the centred stencils, the cube vertices the
 * three-cell mean.  No effect on the doubly periodic grid; other values:
 * FV3_EINVAL. */
typedef struct {
    int kind;            /* fv3_grid_kind                                  */
    int n, nz;           /* cells per tile edge, layers                    */
    double dx, f0;       /* periodic: spacing [m], Coriolis [1/s]          */
    double radius, omega;/* cubed sphere: [m], [1/s]                       */
    double ptop;         /* top pressure [Pa]                              */
    int precision;       /* fv3_precision                                  */
    int hord;            /* PPM order: 8 monotone, 6 unlimited, 5 2dx-filt.*/
    double d2_bg;        /* del-2 divergence damping, 0 (off) .. 0.25      */
    double beta;         /* vertical off-centring, 0.5 .. 1 (1: implicit)  */
    double dddmp;        /* Smagorinsky divergence damping, 0 (off) .. 1   */
    int hord_tr;         /* tracer PPM order: 0 (= hord), 5, 6, 7, 8       */
    int pp_order;        /* interface p' of the column solves: 2 (or 0)
                            mass-linear, 4 cubic                          */
    int nord;            /* higher-order divergence damping: 0 off,
                            1 del-4, 2 del-6                              */
    double d4_bg;        /* its coefficient, 0 .. 0.25                    */
    double vtdm;         /* del-2 vorticity damping, 0 (off) .. 0.25       */
    int edge_fix;        /* cube: edge-flux fix-up, 0 (off) or 1          */
    int edge_ppm;        /* cube: one-sided PPM at tile edges, 0 or 1     */
    int edge_interp;     /* cube: one-sided c_sw / nh_p_grad interpolation
                            at tile edges, 0 or 1                         */
    int device;          /* HIP device ordinal                             */
} fv3_grid_params;

typedef struct fv3_grid fv3_grid;

/* Memory layout of every field.  Element (t, k, j, i) of a field with L
 * levels (L = nz for layer fields, nz + 1 for interface fields, 1 for 2-D
 * fields) sits at
 *     offset0 + (t * L + k) * level_elems + j * pitch + i
 * for i, j in [-halo, n + halo] (index n + halo is used by face and corner
 * staggerings only).  Rows are padded to `pitch` elements and every level is
 * pre-padded so that interior column i = 0 starts on a 128-byte boundary.
 * Staggering (point in units of the grid spacing, tile SW vertex at 0):
 *   cell (i + 1/2, j + 1/2): w, delp, pt, delz, dp0, q, pfull, phi, phis
 *   x-face (i, j + 1/2):     v (D grid), uc (C grid), mfx, cx
 *   y-face (i + 1/2, j):     u (D grid), vc (C grid), mfy, cy
 * A field of L levels needs alloc_elems(L) = offset0 - halo*(pitch + 1)
 * + tiles * L * level_elems + pitch elements. */
typedef struct {
    int tiles, n, nz, halo;
    long pitch, rows, level_elems, offset0;
    int bulk_elem_bytes;   /* 8 for FV3_FP64, 4 for FV3_MIXED */
} fv3_layout;

/* Caller-owned device arrays of one model state.  Bulk-precision fields
 * (u, v, w, delp, pt, uc, vc, cx, cy) are double in FV3_FP64 and float in
 * FV3_MIXED; delz, mfx, mfy, dp0, pfull, phi and phis are always double.
 * `workspace` must hold fv3_workspace_bytes(grid) bytes. */
typedef struct {
    void *u, *v, *w, *delp, *pt;     /* prognostics, updated in place              */
    double *delz;                    /* layer thickness (negative) [m], in place    */
    void *uc, *vc;                   /* C-grid winds (out)                          */
    double *mfx, *mfy;               /* accumulated mass fluxes (out, zeroed)       */
    void *cx, *cy;                   /* accumulated Courant numbers (out, zeroed)   */
    double *dp0;                     /* delp at entry (out)                         */
    double *pfull, *phi;             /* interface pressure [Pa], geopotential (out) */
    const double *phis;              /* surface geopotential (2-D) or NULL = flat   */
    void *workspace;
    size_t workspace_bytes;
    void *qv;                        /* specific humidity [kg/kg] (bulk precision,
                                        cell field) or NULL = dry: the column
                                        solves take theta (1 + (Rv/Rd - 1) qv);
                                        read only, its halo filled at entry    */
} fv3_state;

/* Build a grid on `p->device`: geometry and metric terms (FP64 on the host),
 * tile connectivity by matching shared edges, the halo plan, upload to the
 * device.  Synchronous.  Sec. II (gnomonic cubed sphere); the halo plan
 * carries the orientation transform between adjoining faces of Sec. V-C.
 * Returns FV3_OK and *out, or an error (nothing allocated). */
fv3_status fv3_init_grid(const fv3_grid_params *p, fv3_grid **out);

/* Release a grid (synchronises the device).  NULL is accepted. */
fv3_status fv3_free_grid(fv3_grid *g);

/* Fill *out with the grid's field layout. */
fv3_status fv3_grid_layout(const fv3_grid *g, fv3_layout *out);

/* Bytes of workspace fv3_acoustic_substeps and fv3_tracer_transport need. */
size_t fv3_workspace_bytes(const fv3_grid *g);

/* Copy one metric term of the grid to host memory, as doubles in the field
 * layout with L = 1 (alloc_elems(1) values).  which: 0 dx 1 dy 2 dxc 3 dyc
 * 4 dxa 5 dya 6 area 7 area_c 8 fC 9 fB 10 sin_u 11 cos_u 12 sin_v 13 cos_v
 * 14 sin_a 15 cos_a.  Synchronous. */
fv3_status fv3_grid_metric(const fv3_grid *g, int which, double *host_out);

/* Host-only variant for inspection and tests: compute metric `which` (as
 * in fv3_grid_metric) for the grid `p` on the host, without a device, into
 * host_out as a compact array [tiles][n + 7][n + 7] (row j + 3, column
 * i + 3).  max_elems is the capacity of host_out; FV3_ESHAPE if too small. */
fv3_status fv3_host_grid_metric(const fv3_grid_params *p, int which, double *host_out,
                                long max_elems);

/* Run n_split acoustic substeps of length dt / n_split (the innermost loop
 * of Sec. II): per substep the halo exchange of the D-grid winds and cell
 * fields, c_sw over half a substep, the C-grid vertical solve
 * (riem_solver_c, Sec. IX-B) and pressure gradient, the C-grid wind halo,
 * d_sw with fv_tp_2d transport (Sec. IX-C), riem_solver3, the halo of the
 * interface pressure and geopotential, and the D-grid pressure gradient.
 * On entry mfx, mfy, cx, cy are zeroed and dp0 = delp; they accumulate over
 * the call for fv3_tracer_transport.  Asynchronous on `stream`.
 * Errors: FV3_EINVAL (NULL field, dt not finite or <= 0, n_split < 1,
 * workspace too small). */
fv3_status fv3_acoustic_substeps(fv3_state *s, const fv3_grid *g, double dt, int n_split,
                                 void *stream);

/* Test entry point: as fv3_acoustic_substeps, but in the last substep stop
 * after stage `stop_stage` (1 halo A, 2 c_sw, 3 dz_c + riem_solver_c,
 * 4 p_grad_c, 5 halo B, 6 d_sw, 7 dz_d, 8 riem_solver3, 9 halo C,
 * 10 nh_p_grad = complete).  Used to compare single stages with a
 * reference implementation. */
fv3_status fv3_acoustic_substeps_debug(fv3_state *s, const fv3_grid *g, double dt, int n_split,
                                       int stop_stage, void *stream);

/* Tracer advection of the remapping step (Sec. II) with the fluxes and
 * Courant numbers accumulated by the last fv3_acoustic_substeps on `s`:
 * nsplt sub-cycles (nsplt <= 0: the smallest count that keeps every
 * sub-cycle Courant number <= 1, which costs one device-to-host read), each a
 * halo fill of the tracers and a mass-weighted fv_tp_2d update.  q[m] are
 * device pointers to nq bulk-precision cell fields, updated in place; s->cx
 * and s->cy get their halos filled.  Errors: FV3_EINVAL (NULL pointers,
 * nq < 1 or > 64, nsplt > FV3_MAX_TRACER_SUBCYCLES); with nsplt <= 0,
 * FV3_ENONFINITE when a Courant number is not finite and FV3_ECFL when the
 * count would exceed FV3_MAX_TRACER_SUBCYCLES (nothing is enqueued after
 * the read in either case). */
#define FV3_MAX_TRACER_SUBCYCLES 1024
fv3_status fv3_tracer_transport(void *const *q, int nq, fv3_state *s, const fv3_grid *g,
                                int nsplt, void *stream);

/* Most layers fv3_remap accepts. */
#define FV3_REMAP_MAX_LEVELS 128

/* Vertical remapping of the remapping step (Sec. II): the Lagrangian layers
 * every column has after acoustic substeps are mapped back to the reference
 * interfaces pe_K = ak[K] + bk[K] * ps (K = 0..nz), ps = ptop + the column's
 * sum of delp, by a mass-conserving piecewise-parabolic remap in pressure
 * (Colella-Woodward reconstruction on the non-uniform layers with its
 * monotonicity limiters; constant top and bottom layers).  pt, w and the nq
 * tracer fields q[m] (bulk precision, device) are remapped mass-weighted;
 * delz as delz/delp, so each column keeps its depth; u and v at their faces,
 * with the interface pressures the mean of those of the two cells sharing
 * the face (the halo of delp is filled first); delp becomes the reference
 * thickness.  The column integral of every field times delp is conserved to
 * rounding.  Computes in FP64 in both precision modes.
 * ak, bk: host arrays of nz + 1 doubles, copied into the launch (the call
 * keeps no pointer); ak[0] must equal the grid's ptop, bk[0] = 0, ak[nz] = 0
 * and bk[nz] = 1 exactly.  Uses the state's workspace.  Asynchronous on
 * `stream`.  Errors: FV3_EINVAL (NULL pointers, non-finite or mismatched end
 * coefficients, nq < 0 or > 64), FV3_ESHAPE (nz > FV3_REMAP_MAX_LEVELS);
 * a column whose reference interfaces do not increase latches FV3_EREMAP,
 * reported by fv3_check_status. */
fv3_status fv3_remap(fv3_state *s, const fv3_grid *g, const double *ak, const double *bk,
                     void *const *q, int nq, void *stream);

/* One pass of the remapping loop, the middle of FV3's three nested loops
 * (Sec. II; its share of the run is Table III's "Lagrangian contrib."),
 * over the span dt: k_split times, n_split acoustic substeps of
 * dt / (k_split n_split) (fv3_acoustic_substeps over dt / k_split), then the
 * tracer transport of the nq tracers q[m] with the fluxes those substeps
 * accumulated (fv3_tracer_transport with nsplt; skipped when nq = 0), then the
 * vertical remapping of the state and the tracers to ak + bk ps (fv3_remap).
 * Arguments and their conditions as in those three calls; the accumulators,
 * dp0, pfull and phi hold the last pass's values.  Asynchronous on `stream`
 * except for the sub-cycle count read of each tracer transport when
 * nsplt <= 0.  Errors: those of the three calls (FV3_EINVAL also for
 * k_split < 1); the first failing pass stops the loop. */
fv3_status fv3_dynamics(fv3_state *s, const fv3_grid *g, void *const *q, int nq, const double *ak,
                        const double *bk, double dt, int k_split, int n_split, int nsplt, void *stream);

/* Compensated (Neumaier) FP64 global sums over the interior cells:
 * out[0] = sum delp*area, out[1] = sum pt*delp*area, out[2+m] = sum
 * q[m]*delp*area.  `delp` and `pt` are bulk-precision fields; out is a
 * host array of 2 + nq doubles.  Synchronises `stream`. */
fv3_status fv3_mass_sums(const fv3_grid *g, const void *delp, const void *pt, void *const *q,
                         int nq, double *host_out, void *stream);

/* Size of the fixed device scratch of fv3_mass_sums_noalloc: 4 MiB per GPU,
 * held from the first fv3_init_grid on that GPU until the process ends. */
#define FV3_NOALLOC_SCRATCH_BYTES (4u << 20)

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same sums as
 * fv3_mass_sums, with no device or host allocation and no synchronisation.
 * The per-block partials go to a fixed device array of
 * FV3_NOALLOC_SCRATCH_BYTES instead of the grid's reduction buffer, and are
 * combined on the device in the same order and with the same compensated
 * additions, so the results are bit-identical to fv3_mass_sums.
 * dev_out: DEVICE array of 2 + nq doubles (caller-owned), written
 * asynchronously on `stream` in fv3_mass_sums' order.  Every call on one GPU
 * shares that GPU's scratch array: calls that overlap on one GPU (on
 * different streams or host threads) race and give wrong sums; calls in
 * stream order are safe (each fully overwrites the partials it reads).
 * Errors: FV3_EINVAL (NULL pointers, nq outside 0..64), FV3_EDEVICE (the
 * current device is not the grid's), FV3_ESHAPE (the grid needs more block
 * partials than the scratch holds: 2 doubles per 64 x 4 block of every tile,
 * which fits any doubly periodic tile and cubes up to about C3300). */
fv3_status fv3_mass_sums_noalloc(const fv3_grid *g, const void *delp, const void *pt, void *const *q,
                                 int nq, double *dev_out, void *stream);

/* Fill the halos of n_fields cell-centred fields (L levels each, bulk
 * precision unless fp64 != 0) from the neighbouring tiles.  Exposed for
 * tests of the halo exchange. */
fv3_status fv3_halo_fill(const fv3_grid *g, void *const *fields, int n_fields, int levels,
                         int fp64, void *stream);

/* Synchronise `stream`, then return and clear the first device-detected
 * error latched on the grid (FV3_ECFL, FV3_ENONFINITE, FV3_EREMAP) or
 * FV3_OK. */
fv3_status fv3_check_status(const fv3_grid *g, void *stream);

/* Measurement support.  fv3_timing_start(filter) makes every later kernel
 * launch of the library whose kernel name contains `filter` ("" = all) record
 * a pair of HIP events on its stream; fv3_timing_stop() stops recording,
 * synchronises the device and reports, per distinct kernel name (up to cap),
 * the total elapsed milliseconds and the number of launches.  Kernel names
 * are written NUL-separated into `names` (names_cap bytes).  Returns the
 * number of kernels reported, or a negative fv3_status.  Not thread-safe. */
fv3_status fv3_timing_start(const char *filter);
/* Measurement support: copy `bytes` (a multiple of 16, both addresses
 * 16-byte aligned, no overlap) from device memory src to dst with the
 * library's streaming copy kernel (16-byte accesses), the practical HBM roof
 * that kernel timings are set against.  Asynchronous on `stream`; timed as
 * "k_stream_copy".  Errors: FV3_EINVAL. */
fv3_status fv3_device_copy(const void *src, void *dst, size_t bytes, void *stream);
int fv3_timing_stop(char *names, int names_cap, double *total_ms, long *counts, int cap);

const char *fv3_status_string(fv3_status s);
const char *fv3_last_error(void);

/* ------------------------------------------------------------------------
 * Batched ensemble of independent grids.  The paper tunes one program
 * across many stencil instances and reuses the tuning where the same
 * pattern recurs (transfer tuning, Sec. VII-B); it runs one model per
 * allocation.  Here many small, uneven members share one GPU: every kernel
 * of the substep sequence runs once for all members (member-indexed blocks,
 * per-member arguments in device memory), optionally replayed from a HIP
 * graph, with block shapes chosen by timing and reused per kernel.
 * ------------------------------------------------------------------------ */

/* Run n_split acoustic substeps of dt / n_split on each of `members`
 * (state, grid) pairs, exactly as fv3_acoustic_substeps would on each alone
 * (same kernels, bit-identical results), with one launch per kernel for all
 * members.  All grids must share one precision and be on the current device
 * (else FV3_EDTYPE / FV3_EDEVICE), and the options that choose kernels: PPM
 * orders, damping switches, off-centring, the tile-edge options and humidity
 * (a member whose launch sequence differs from the first member's:
 * FV3_EUNSUPPORTED).  Grid kinds and sizes may differ.
 * Convenience form: builds an ensemble, runs it and synchronises `stream`. */
fv3_status fv3_acoustic_substeps_batched(fv3_state *const *states, const fv3_grid *const *grids,
                                         int members, double dt, int n_split, void *stream);

typedef struct fv3_ensemble fv3_ensemble;
enum { FV3_ENSEMBLE_GRAPH = 1 };   /* replay the whole call from a captured HIP graph */

/* Record the substep launch sequence of every member (host only, nothing
 * runs) and upload the per-member argument tables.  The states, grids and
 * their device arrays must outlive the ensemble; each fv3_ensemble_run is
 * one call of n_split substeps of dt / n_split on every member. */
fv3_status fv3_ensemble_create(fv3_state *const *states, const fv3_grid *const *grids, int members,
                               double dt, int n_split, int flags, fv3_ensemble **out);
fv3_status fv3_ensemble_run(fv3_ensemble *e, void *stream);   /* asynchronous */
fv3_status fv3_ensemble_free(fv3_ensemble *e);                /* synchronises the device */

/* Autotuner report: plane kernels (tunable sites) whose block shape was
 * searched by timing `reps` launches of each candidate shape, and those that
 * reused a shape found earlier for the same kernel (at another stage of the
 * sequence, or by an earlier ensemble in this process); search time; one
 * substep's time before and after. */
typedef struct {
    int sites, tunable_sites, searched, reused;
    double search_ms, substep_ms_before, substep_ms_after;
} fv3_tune_report;

/* Choose block shapes by timing.  Runs kernels of the sequence repeatedly on
 * the ensemble's states, which are left in an undefined state: tune on
 * scratch copies, then reload.  Synchronous. */
fv3_status fv3_ensemble_tune(fv3_ensemble *e, int reps, fv3_tune_report *report, void *stream);

/* Inspection: kernel names (NUL-separated) and block shapes of the recorded
 * sequence; returns the number of sites written. */
int fv3_ensemble_shapes(const fv3_ensemble *e, char *names, int names_cap, int *block_x,
                        int *block_y, int cap);

/* ------------------------------------------------------------------------
 * Learned per-column correction of a coarse run.  The paper motivates
 * coupling machine-learned components with the dynamical core (Sec. III)
 * without giving a recipe; the entry points below are this library's
 * recipe: coarsen a fine run, extract normalised column features, train a
 * three-layer perceptron with BF16 matrix-core products and FP32
 * accumulation, and add its predicted tendencies to a coarse state.
 * ------------------------------------------------------------------------ */

/* Coarsen u, v, w, delp, pt and delz of `fine` (grid gf) onto `coarse`
 * (grid gc) with gf->n = r * gc->n for an integer r >= 1, same tiles, levels
 * and precision.  Cell values: delp and delz are area means of the r x r
 * fine cells, pt and w mass-weighted (delp * area) means.  D-grid winds: the
 * edge-length-weighted mean of the r fine edges on each coarse edge, which
 * keeps the circulation along it.  Halos of `coarse` are not filled.
 * Asynchronous.  Errors: FV3_EINVAL (NULL), FV3_ESHAPE (sizes), FV3_EDTYPE
 * (precisions differ). */
fv3_status fv3_coarsen(const fv3_state *fine, const fv3_grid *gf, fv3_state *coarse,
                       const fv3_grid *gc, void *stream);

/* Per-feature normalisation, device arrays of 5 * nz floats, feature order
 * (field, level) with fields ua, va, pt, w, delp: z = (x - mean) * inv_std.
 * lo and hi are the training range of z; they may be NULL when no flag is
 * requested. */
typedef struct {
    const float *mean, *inv_std, *lo, *hi;
} fv3_feature_norm;

/* Column features of every interior column into X, a device float array of
 * (tiles * n * n) rows (order tile, j, i) by 5 * nz columns, row-major.  ua
 * and va are the means of the two D-grid faces of each cell (tile
 * components).  If `flag` (device int) is not NULL, bit 0 is set when any z
 * is not finite or lies more than 6 outside [lo, hi]; the flag is only ever
 * set, never cleared.  Asynchronous. */
fv3_status fv3_column_features(const fv3_state *s, const fv3_grid *g, const fv3_feature_norm *norm,
                               float *X, int *flag, void *stream);

/* Add `seconds` times the tendencies Y (device, rows as fv3_column_features,
 * 3 * nz columns: ua, va, pt; normalised, physical = Y * ystd + ymean) to
 * the state: pt in place; the cell wind increments are exchanged across tile
 * edges and each D-grid face takes the mean of its two cells.  Bit 1 of
 * *flag (device int) is set if any Y is not finite; when *flag is nonzero
 * after that check (including bits set earlier by fv3_column_features) the
 * state is left unchanged -- the plain coarse run is the fallback.  Uses the
 * first 2 * alloc_elems(nz) doubles of s->workspace.  Asynchronous. */
fv3_status fv3_apply_correction(fv3_state *s, const fv3_grid *g, const float *Y, const float *ymean,
                                const float *ystd, double seconds, int *flag, void *stream);

/* Three-layer perceptron x -> tanh(x W1 + b1) -> tanh(. W2 + b2) -> . W3 + b3
 * on the current HIP device.  Matrix products take BF16 operands (round to
 * nearest even) on the matrix cores with FP32 accumulation; parameters,
 * Adam moments and activations' derivatives are FP32.  Hidden widths must be
 * multiples of 16; input and output widths are padded to 16 internally.
 * `params` (host) are packed as W1 (in x h1, row-major), b1, W2, b2, W3, b3;
 * rows <= maxrows for every call. */
typedef struct fv3_mlp fv3_mlp;
fv3_status fv3_mlp_create(int in, int h1, int h2, int out, int maxrows, const float *params,
                          fv3_mlp **net);
fv3_status fv3_mlp_free(fv3_mlp *net);
long fv3_mlp_param_count(const fv3_mlp *net);
/* replace the parameters (host, packed) and reset the Adam state; synchronous */
fv3_status fv3_mlp_set_params(fv3_mlp *net, const float *params);
/* copy the FP32 master parameters to host (packed); synchronous */
fv3_status fv3_mlp_get_params(const fv3_mlp *net, float *params);
/* Y (device, rows x out) = network(X (device, rows x in)); asynchronous */
fv3_status fv3_mlp_forward(fv3_mlp *net, const float *X, int rows, float *Y, void *stream);
/* Gradients of the mean squared error mean((Y - T)^2) over rows x out with
 * respect to the parameters, packed as `params`, to host; synchronous. */
fv3_status fv3_mlp_gradients(fv3_mlp *net, const float *X, const float *T, int rows, float *grads,
                             void *stream);
/* One Adam step (betas 0.9, 0.999, eps 1e-8, learning rate lr) on the batch
 * X, T (device).  If loss is not NULL the batch loss before the step is
 * written there (synchronises `stream`); otherwise asynchronous. */
fv3_status fv3_mlp_train_step(fv3_mlp *net, const float *X, const float *T, int rows, float lr,
                              double *loss, void *stream);

#ifdef __cplusplus
}
#endif

#endif
