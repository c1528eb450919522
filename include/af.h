/*
 * af.h -- C ABI of the MI355X (gfx950) Active Flux library libaf.so.
 *
 * The library advances the fully discrete third-order Active Flux method for the 2D Euler
 * equations on a Cartesian grid (Chudzik, Helzel, Porfetye, arXiv 2508.06273):
 *   - point values at cell corners and edge midpoints are evolved to the intermediate and the
 *     new time level with the EG2 bicharacteristic evolution operator of the locally
 *     linearised system plus the correction term of Corollary 1 (Sec. 2, Algorithm 1; the
 *     averaged linearisation of Sec. 3.1; the simplified method, eq. 1stStep);
 *   - cell averages are updated conservatively with Simpson space-time fluxes
 *     (Sec. 2, eqs. 2dfvm and F);
 *   - optionally, point values with negative density or pressure are replaced by EG1 on
 *     piecewise constant data and, failing that, by a Lax-Friedrichs update (Algorithm 3),
 *     and face fluxes are limited so that the cell averages stay admissible (Sec. 3.5);
 *   - boundaries are periodic, outflow (piecewise constant extrapolation, Sec. 4), solid wall
 *     or inflow (Sec. 4.3), chosen per side.
 *
 * Degrees of freedom and host array layout (all host arrays are FP64, variable-major,
 * unpadded, C order):
 *   avg : 4 x ny x nx            conserved cell averages (rho, rho u, rho v, E)
 *   K   : 4 x nky x nkx          primitive (rho, u, v, p) at corners (x0 + i dx, y0 + j dy)
 *   X   : 4 x ny  x nkx          primitive at vertical-edge midpoints (x0 + i dx, y0 + (j+1/2) dy)
 *   Y   : 4 x nky x nx           primitive at horizontal-edge midpoints (x0 + (i+1/2) dx, y0 + j dy)
 * with nkx = nx + (x periodic ? 0 : 1), nky = ny + (y periodic ? 0 : 1).  The ideal gas law
 * E = p/(gamma-1) + rho (u^2 + v^2)/2 links the two sets of variables.
 *
 * Ownership: the caller owns every host array; the library copies in and out synchronously on
 * the handle's stream and keeps no pointer.  Device memory belongs to the handle.
 * Errors: every call returns AF_OK (0) or a negative code; af_last_error() gives the text.
 * A step that fails leaves the state at the beginning of that step; if several degrees of
 * freedom fail in one step, AF_ERR_CFL is reported before AF_ERR_NONPHYSICAL.  A handle is not
 * thread-safe; different handles are independent.  The library needs a gfx950 GPU: without
 * one, af_create returns AF_ERR_DEVICE.
 */
#ifndef AF_H
#define AF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct af_handle af_handle;

/* Grid: nx x ny cells covering [x0,x1] x [y0,y1]; dx = (x1-x0)/nx, dy = (y1-y0)/ny. */
typedef struct {
  int32_t nx, ny;
  double x0, x1, y0, y1;
} af_grid;

/* Boundary condition per side (Sec. 4 and 4.3).  Periodic must be set on both sides of an
 * axis.  The DOFs on a non-periodic boundary line are evolved like interior ones; the data
 * beyond the side (one layer of ghost cells and their point values) are:
 *   AF_BC_OUTFLOW : copies of the nearest boundary cell average / point value;
 *   AF_BC_WALL    : the mirror image about the boundary line of the interior at the same
 *                   distance, with the normal velocity (and momentum) negated: ghost point
 *                   values are the reflected point values, a ghost cell is the reflection
 *                   of the cell it faces (average, reconstruction, centre value).  With
 *                   AF_LIN_AVG a DOF on a wall line is linearised at its own point value
 *                   instead of the mean of the adjacent averages;
 *   AF_BC_INFLOW  : the side's inflow state (af_set_inflow) for every ghost point value, the
 *                   ghost cells' centre values included.
 * Beyond a domain corner the walls' reflections apply first, then an inflow side's state
 * replaces the value (the y side's if both sides are inflow). */
enum { AF_BC_PERIODIC = 0, AF_BC_OUTFLOW = 1, AF_BC_WALL = 2, AF_BC_INFLOW = 3 };
typedef struct {
  int32_t left, right, bottom, top;
} af_bc;
/* Side numbers of af_set_inflow. */
enum { AF_SIDE_LEFT = 0, AF_SIDE_RIGHT = 1, AF_SIDE_BOTTOM = 2, AF_SIDE_TOP = 3 };

enum {
  AF_OK = 0,
  AF_ERR_INVALID_ARG = -1, /* bad handle, size, option or argument */
  AF_ERR_NONPHYSICAL = -2, /* non-positive density or pressure where the method needs it */
  AF_ERR_CFL = -3,         /* an evolution circle would leave the cells around its point */
  AF_ERR_DEVICE = -4,      /* HIP runtime error or no usable GPU */
  AF_ERR_OOM = -5          /* device allocation failed */
};

/* Options (af_set_option).  They apply from the next step on; the state is kept. */
enum {
  AF_OPT_PRECISION = 1,     /* AF_PREC_FP64 (default) or AF_PREC_FP32 (see below)        */
  AF_OPT_LINEARISATION = 2, /* AF_LIN_AF3 (default), AF_LIN_AVG or AF_LIN_SIMPLE          */
  AF_OPT_CORRECTION = 3,    /* 1 (default): add C of Corollary 1; 0: drop it              */
  AF_OPT_LIMITER = 4,       /* 0 (default): none; 1: bound-preserving point values (Alg.3)*/
  AF_OPT_GRAPH_STEPS = 5,   /* steps per captured HIP graph in af_run (even, 0 = no graph) */
  AF_OPT_TIMING = 6,        /* 1: launch eagerly and time every kernel with HIP events on the
                               handle's stream (af_get_timing); 0 (default): off           */
  AF_OPT_AUTOTUNE = 7,      /* batched handles: 1 = the next af_run times, on its first
                               steps (2 steps each), every tile order and update workgroup
                               size with separate kernels and every tile order with the
                               persistent step kernel, and keeps the fastest schedule; the
                               results do not depend on the schedule.  0 (default): keep the
                               current schedule.  No effect on single-grid handles.       */
  AF_OPT_TILE_ORDER = 8,    /* batched handles: order in which the point kernel's workgroups
                               take the tiles of all grids (AF_ORDER_*; default XCD)      */
  AF_OPT_UPDATE_THREADS = 9, /* batched handles: workgroup size of the update kernel, one
                               row of cells per workgroup: 64, 128 (default) or 256        */
  AF_OPT_TRANSONIC = 10,    /* 1: Algorithm 2.  A corner is flagged when, across its two
                               rows (columns) of cells, u + c or u - c (v + c or v - c) of
                               the primitive averages goes from positive to negative; a
                               flagged corner, or an edge midpoint with a flagged end
                               corner, linearises its new time level at the mean of the
                               adjacent primitive averages instead of U^{n+1/2}.  Meant
                               with AF_LIN_AVG (Sec. 3.1).  0 (default): off.              */
  AF_OPT_SHOCK_LIMITER = 11,/* 1: shock-indicator limiting of point values (Sec. 3.4): the
                               intermediate and the new value become theta U + (1 - theta)
                               U_lo, U_lo being EG1 on piecewise constant data linearised at
                               the mean of the adjacent primitive averages (as in
                               Algorithm 3), theta = exp(-phi1 phi2), phi1 the larger of the
                               two pressure sensors |p(k+1) - 2p(k) + p(k-1)| / (p(k+1) +
                               2p(k) + p(k-1)) centred on the two cells next to an edge
                               midpoint, phi2 = 2^max(|w| + c) over those cells (w: the
                               velocity along the edge normal); a corner takes the smallest
                               theta of its four edges.  A non-admissible average in a
                               sensor's stencil gives theta = 0; where the mean of the
                               averages is not admissible the value is not blended.
                               Algorithm 3 (AF_OPT_LIMITER) then runs on the blended value.
                               0 (default): off.                                          */
  AF_OPT_FLUX_LIMITER = 12, /* 1: flux limiting of the cell averages (Sec. 3.5): every face
                               flux becomes gamma F + (1 - gamma) F_lo, F the Simpson flux,
                               F_lo the Rusanov flux of the t_n averages of the two cells,
                               gamma in [0, 1] the smaller over the two cells of the largest
                               theta that keeps the cell's share Q_lo - 4 (dt/h) s theta
                               (F - F_lo) of its new average at density and pressure of at
                               least min(1e-13, those of its low-order update Q_lo) (after
                               Hu, Adams and Shu, 2013).  The new averages are then
                               admissible whenever the low-order updates are.  Faces need
                               no limiting in smooth flow (gamma = 1: the unlimited step,
                               bit for bit).  Single-grid handles.  0 (default): off.      */
  AF_OPT_STEP_KERNEL = 13,  /* batched handles: AF_STEP_SPLIT (default) launches the point,
                               fix-up, update and commit kernels in turn; AF_STEP_PERSISTENT
                               runs the whole step in one launch of a persistent kernel: as
                               many workgroups as the GPU holds at once take the step's work
                               (indicator rows, tiles, listed tiles, update chunks) from
                               device-side queues, phase after phase, with grid-wide barriers
                               between the phases, and the last to finish commits every grid.
                               A barrier not reached within 2 s (workgroups not all resident,
                               e.g. another kernel sharing the GPU) ends the step of every
                               running grid with AF_ERR_DEVICE, the state kept at t_n
                               (the limit: AF_OPT_SYNC_TIMEOUT_US).                       */
  AF_OPT_SYNC_TIMEOUT_US = 14 /* batched handles: how long a workgroup of the persistent step
                               kernel waits at a barrier before the step is abandoned, in
                               microseconds of the GPU's wall clock, 0 .. 1e8 (default 2e6;
                               0: the step ends with AF_ERR_DEVICE unless every workgroup
                               is already there).                                          */
};
/* Tile orders of the batched point kernel.  Workgroups are dealt to the GPU's 8 XCDs in turn;
 * AF_ORDER_XCD gives each XCD a contiguous range of the global tile index, AF_ORDER_LINEAR
 * takes the tiles in index order, AF_ORDER_GRIDS packs whole grids onto the XCDs. */
enum { AF_ORDER_XCD = 0, AF_ORDER_LINEAR = 1, AF_ORDER_GRIDS = 2 };
/* Step kernels of batched handles (AF_OPT_STEP_KERNEL). */
enum { AF_STEP_SPLIT = 0, AF_STEP_PERSISTENT = 1 };
/* AF_PREC_FP64: every operation in FP64.  AF_PREC_FP32 (FP32 bulk): the evolution operators
 * (moment recurrences, circle shifts and contractions of EG2 and EG1) and the correction term
 * run in FP32 on deviations from the linearisation state; point values and cell averages are
 * stored in FP64, the deviations themselves, the state updates, the Simpson fluxes and the
 * average update, the positivity tests and the time step are FP64. */
enum { AF_PREC_FP64 = 0, AF_PREC_FP32 = 1 };
/* AF_LIN_AF3: Algorithm 1 (intermediate values linearised at EG2(U^n, dt/4));
 * AF_LIN_AVG: intermediate values linearised at the mean of the adjacent primitive cell
 *             averages (Sec. 3.1, eq. Un+1/2);
 * AF_LIN_SIMPLE: intermediate values linearised at U^n (eq. 1stStep).
 * In every mode the new time level is linearised at the intermediate value. */
enum { AF_LIN_AF3 = 0, AF_LIN_AVG = 1, AF_LIN_SIMPLE = 2 };

/* Counters returned by af_get_counters (cumulative since af_set_state). */
enum {
  AF_CNT_EG1 = 0,        /* point values replaced by EG1 on piecewise constant data   */
  AF_CNT_LF = 1,         /* point values replaced by the Lax-Friedrichs update        */
  AF_CNT_CENTRE = 2,     /* cells whose inverse-Simpson centre value was not admissible
                            and fell back to the primitive value of the average        */
  AF_CNT_INNER = 3,      /* Algorithm 1 inner states not admissible (the intermediate
                            value was then linearised at U^n)                          */
  AF_CNT_STEPS = 4,      /* steps taken                                               */
  AF_CNT_TSW = 5,        /* DOFs whose new time level took the transonic-shock
                            linearisation (AF_OPT_TRANSONIC)                           */
  AF_CNT_FLUX = 6,       /* faces whose flux was limited (AF_OPT_FLUX_LIMITER)        */
  AF_NCOUNTERS = 8
};

/* Create a solver for `grid` with ratio of specific heats `gamma` (> 1) and boundary
 * conditions `bc` (Sec. 2: the Cartesian grid of cells with averages at the centres and point
 * values at the corners and edge midpoints; the ideal gas law with gamma; Sec. 4 and 4.3: the
 * boundary kinds).  Allocates the device state (uninitialised until af_set_state).  `out`
 * receives the handle, owned by the caller until af_destroy.  Errors: AF_ERR_INVALID_ARG for
 * nx or ny outside [2, 65536], non-finite or empty domain bounds, a cell size that is not a
 * finite positive number (below 1e-150), gamma not finite or <= 1, an unknown boundary kind
 * or a periodic side without its partner (all checked before any HIP call);
 * AF_ERR_DEVICE without a usable GPU; AF_ERR_OOM. */
int af_create(const af_grid* grid, double gamma, const af_bc* bc, af_handle** out);

/* Set an option (keys and values above; each key names the passage whose variant it selects:
 * Algorithm 1/eq. Un+1/2/eq. 1stStep, Corollary 1, Algorithms 2 and 3, Secs. 3.4 and 3.5).
 * Errors: AF_ERR_INVALID_ARG for an unknown key or value. */
int af_set_option(af_handle* h, int key, int64_t value);

/* Current value of an option (for AF_OPT_TILE_ORDER and AF_OPT_UPDATE_THREADS after an
 * autotuned run: the schedule the tuner kept).  The tile order and update threads are
 * AF_ERR_INVALID_ARG on single-grid handles.  Runtime control; no passage of the paper. */
int af_get_option(const af_handle* h, int key, int64_t* value);

/* Use `hip_stream` (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream) for all
 * device work of this handle.  NULL selects the handle's own (non-blocking) stream.  Runtime
 * plumbing; no passage of the paper. */
int af_set_stream(af_handle* h, void* hip_stream);

/* Copy a state in (host FP64 arrays, layout above) at time t: the conserved cell averages and
 * the primitive point values that are the method's degrees of freedom (Sec. 2, the start of a
 * step t_n).  Resets the counters.  The arrays stay the caller's.  Errors: AF_ERR_INVALID_ARG
 * (NULL array, t not finite), AF_ERR_NONPHYSICAL if an average has rho <= 0 or p <= 0 (the
 * state is then not set). */
int af_set_state(af_handle* h, const double* avg, const double* K, const double* X,
                 const double* Y, double t);

/* Copy the current state out (the degrees of freedom of Sec. 2 at the current time; any output
 * pointer may be NULL).  Errors: AF_ERR_INVALID_ARG if no state was set. */
int af_get_state(const af_handle* h, double* avg, double* K, double* X, double* Y,
                 double* t);

/* One time step of size dt > 0 (Algorithm 1 steps 1-3 with the chosen options). */
int af_step(af_handle* h, double dt);

/* Advance to t_end with dt = cfl * min(dx,dy) / max over all DOFs of (max(|u|,|v|) + c)
 * (the CFL number of Sec. 2, which states stability of the linear schemes up to 0.279),
 * computed on the device from the current state before every step; the last step is cut
 * to land on t_end.  max_steps > 0 bounds the number of steps.  t_reached and steps_taken
 * (nullable) report where the run stopped.  Errors: AF_ERR_INVALID_ARG for cfl outside
 * (0, 0.5) or a NaN t_end; a failing step ends the run with its code (the state is then the
 * one before that step, t_reached and steps_taken say where). */
int af_run(af_handle* h, double t_end, double cfl, int64_t max_steps, double* t_reached,
           int64_t* steps_taken);

/* Counters (AF_NCOUNTERS values, indices AF_CNT_*): how often Algorithm 3's low-order
 * branches, the centre-value fallback, the Algorithm 1 inner-state fallback, Algorithm 2 and
 * the flux limiting of Sec. 3.5 acted, and the steps taken.  `out` is the caller's. */
int af_get_counters(const af_handle* h, int64_t* out);

/* Free the handle and its device memory (NULL is ignored).  Runtime plumbing. */
void af_destroy(af_handle* h);

/* Domain totals of the conserved variables of the current state of grid g (0 on a single-grid
 * handle): out[0..3] = the sums over the grid's cells of the averages of rho, rho u, rho v and
 * E, times the cell area -- the quantities the conservative update (eq. 2dfvm) keeps on a
 * periodic grid.  Computed on the device in FP64 by a reduction in a fixed order (the same
 * bits for the same state), synchronous on the handle's stream; out is the caller's (4
 * doubles).  For conservation checks and per-step monitoring between af_step calls.  Errors:
 * AF_ERR_INVALID_ARG (NULL argument, bad grid index, no state set). */
int af_get_totals(const af_handle* h, int32_t g, double* out);

/* Text of the last error on this handle (or of the last failed af_create if h is NULL).
 * Runtime plumbing; the errors of the method are those of Algorithm 3 and of the CFL
 * condition of Sec. 2 (AF_ERR_NONPHYSICAL, AF_ERR_CFL). */
const char* af_last_error(const af_handle* h);

/* Number of DOF sites (averages + K + X + Y) of the handle's grid -- the degrees of freedom of
 * Sec. 2: a cell average per cell, point values at the corners and edge midpoints -- the unit
 * of the DOF-updates/s throughput figure. */
int64_t af_dof_count(const af_handle* h);

/* Measurement, no passage of the paper.  Kernel times gathered while AF_OPT_TIMING is on,
 * summed since the option was last set:
 * out[0] = milliseconds in the point-value kernel, out[1] = milliseconds in the flux/update
 * kernel, out[2] = number of steps timed: those in which a grid advanced (launches that a
 * batched run enqueues after all its grids have stopped are not counted).  Both kernels run on
 * the handle's stream. */
int af_get_timing(const af_handle* h, double* out);

/* ---------------------------------------------------------------------------------------
 * Batched grids: many independent grids (own sizes, domains, boundaries, time steps) in one
 * handle, advanced together with one launch of each kernel per step for all grids, or with one
 * launch of a persistent kernel per step (AF_OPT_STEP_KERNEL).  This is
 * the method of Sec. 2 applied to each grid independently; nothing couples the grids.
 * Options, af_set_stream, af_step, af_run, af_get_counters, af_get_timing, af_dof_count,
 * af_last_error and af_destroy work on batched handles as on single ones:
 *   af_step(dt)  steps every grid with the same dt; a grid whose step fails keeps its state,
 *                the others advance; the most negative error code is returned, its text
 *                names the grid;
 *   af_run       gives every grid its own dt from its own wave speeds; each grid stops at
 *                t_end or after max_steps of its own steps; t_reached is the smallest time
 *                over the grids, steps_taken the largest number of steps;
 *   af_get_counters sums the counters over the grids (AF_CNT_STEPS: the largest).
 * af_set_state / af_get_state work only when n == 1; use the _grid variants.
 * --------------------------------------------------------------------------------------- */

/* Create a handle for n >= 1 grids: grids[g], bcs[g] as for af_create (Sec. 2's grid and
 * DOFs, Sec. 4.3's sides, per grid), one gamma.  Errors as for af_create. */
int af_create_batch(int32_t n, const af_grid* grids, double gamma, const af_bc* bcs,
                    af_handle** out);

/* Number of grids of the handle (1 for af_create handles; 0 for NULL).  Runtime plumbing. */
int32_t af_batch_size(const af_handle* h);

/* af_set_state / af_get_state for grid g (0 <= g < n; g = 0 on single handles): the DOFs of
 * Sec. 2 of that grid at its t_n.  Arrays as for one grid of grids[g]'s sizes.  Every grid
 * needs a state before af_step or af_run.  Errors as for af_set_state / af_get_state, and
 * AF_ERR_INVALID_ARG for a bad grid index. */
int af_set_state_grid(af_handle* h, int32_t g, const double* avg, const double* K,
                      const double* X, const double* Y, double t);
int af_get_state_grid(const af_handle* h, int32_t g, double* avg, double* K, double* X,
                      double* Y, double* t);

/* Time t_n and steps taken (since af_set_state_grid) of grid g in its own time stepping
 * (Sec. 2: dt from the CFL condition of its own state); nullable outputs.  Errors:
 * AF_ERR_INVALID_ARG for a bad grid index. */
int af_get_grid_info(const af_handle* h, int32_t g, double* t, int64_t* steps);

/* The DOFs of Sec. 2, as af_set_state_grid / af_get_state_grid, for arrays in device memory
 * of the handle's GPU (for
 * instance torch tensors), in the host layout above (FP64, variable-major, unpadded): copied
 * device to device on the handle's stream, synchronously, with no host staging; the caller
 * keeps ownership.  The averages are checked on the device (AF_ERR_NONPHYSICAL if one is not
 * admissible).  g = 0 on single-grid handles.  Output pointers may be NULL. */
int af_set_state_device(af_handle* h, int32_t g, const double* avg, const double* K,
                        const double* X, const double* Y, double t);
int af_get_state_device(const af_handle* h, int32_t g, double* avg, double* K, double* X,
                        double* Y, double* t);

/* Inflow state W = (rho, u, v, p) (primitive, rho > 0, p > 0; copied) of side `side`
 * (AF_SIDE_*) of grid g (0 on single handles), which must have been created AF_BC_INFLOW
 * (Sec. 4.3).  Every inflow side needs its state before af_step or af_run
 * (AF_ERR_INVALID_ARG otherwise); it applies from the next step on and may be changed
 * between steps. */
int af_set_inflow(af_handle* h, int32_t g, int32_t side, const double* W);

/* ---------------------------------------------------------------------------------------
 * One step that allocates nothing, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The same step as
 * af_step (same kernels and arithmetic, no indicator options), on caller-owned device arrays
 * in the library's device layout:
 *   avg_in/avg_out : 4 x ny rows x pitch_avg doubles (variable v at v * ny * pitch_avg);
 *   K, X, Y (in/out): 4 x nky rows x pitch_pts doubles each (variable v at v * nky * pitch_pts;
 *                    X uses the first ny rows of each variable),
 * nkx, nky as above; pitches even, pitch_avg >= nx, pitch_pts >= nkx; every pointer 16-byte
 * aligned; no output may alias an input.  `inflow` (host, 4 x 4, row = side, nullable unless a
 * side is AF_BC_INFLOW) gives the inflow states.  Options as AF_OPT_PRECISION,
 * AF_OPT_LINEARISATION, AF_OPT_CORRECTION and AF_OPT_LIMITER.  Work is enqueued on `stream`
 * (a hipStream_t; NULL: the null stream) and the call waits for it; `counters` (host, nullable,
 * AF_NCOUNTERS values) receives this step's counters.
 * Scratch: step control, the grid descriptor, fix-up masks and the per-site flux sums live in a
 * static device array
 * of 32 MiB per GPU (held until the process ends): grids whose flux sums (128 bytes per
 * nky * pitch_pts site) and tile masks do not fit, about 500 x 500 cells, are rejected with
 * AF_ERR_INVALID_ARG.  Every call on one GPU uses that GPU's array: calls that overlap on one
 * GPU (several host threads or streams) race.  No hipMalloc, hipFree or allocating routine is
 * called.  Errors as af_step (the outputs are then unspecified, the inputs unchanged); the text
 * is af_last_error(NULL). */
int af_step_noalloc(const af_grid* grid, double gamma, const af_bc* bc, const double* inflow,
                    int32_t precision, int32_t linearisation, int32_t correction,
                    int32_t limiter, const double* avg_in, const double* K_in,
                    const double* X_in, const double* Y_in, double* avg_out, double* K_out,
                    double* X_out, double* Y_out, int64_t pitch_avg, int64_t pitch_pts,
                    double dt, void* stream, int64_t* counters);

#ifdef __cplusplus
}
#endif
#endif
