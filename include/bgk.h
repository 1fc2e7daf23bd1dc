/*
 * bgk.h -- C ABI of the MI355X BGK discrete-velocity stepper (libbgk.so).
 *
 * The library advances the distribution function f(x, v) of the BGKW model
 * kinetic equation (Frezzotti, Ghiroldi and Gibelli, "Solving Kinetic
 * Equations on GPUs I: Model Kinetic Equations", arXiv:0903.4044, Sec. 2,
 * Eq. (BGKW)) on a spatial grid times a uniform 3D velocity grid (Sec. 2.1),
 * for the paper's two problems: the 1D normal shock (Sec. 4.1) and the 2D
 * lid-driven cavity with diffuse walls (Sec. 5.1), its extension to a
 * lid-driven cube (Sec. 2.1: one upwind stencil per spatial direction), plus
 * periodic test boxes.
 *
 * One time step is R_{dt/2} S_dt R_{dt/2} (Strang) or R_dt S_dt (Lie, the
 * order of Sec. 2.1), where R_tau is the exact homogeneous relaxation of
 * Eq. (relaxation) towards the local Maxwellian of Eq. (Maxw), built from the
 * moments of Eq. (macroscopic) of R's own input, and S_dt is free streaming
 * (Eq. freestreaming) by a minmod-limited upwind scheme in flux form whose
 * first-order special case is Eq. (upwind).
 *
 * Units are those of Sec. 4.1: velocity in sqrt(2 R T_r), so the Maxwellian
 * is n (pi T)^(-3/2) exp(-|v - V|^2 / T) and the collision frequency of
 * Eq. (frequency) with mu ~ T^omega is nu = n T^(1 - omega) / Kn.
 *
 * Memory.  All arrays passed to the calls below are DEVICE pointers owned by
 * the caller (typically torch tensors).  f holds every instance of the
 * context back to back; instance k starts at element f_offset(k) and is
 * laid out f[cell][jz][jy][jx] (velocity fastest, jx fastest of all;
 * cell = (iz * ny + iy) * nx + ix).  Elements are double for BGK_FP64 and float for
 * BGK_FP32.  Every buffer the size of f is the caller's: besides f and its
 * output, bgk_step takes a workspace of ws_step_bytes (its ping-pong
 * buffer) and bgk_step_adjoint one of ws_adjoint_bytes (two f-sized
 * intermediate states), both reported by bgk_sizes.  The context owns only
 * small per-cell and per-instance device data (table entries of the
 * Maxwellians, moment partial sums, the reverse sweep's per-cell
 * coefficients, the rounding counter), allocated in bgk_init and at the
 * first reverse-sweep or lid-shear call.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the default
 * stream).  Work is enqueued asynchronously; no call below synchronises the
 * host except bgk_check, bgk_timing and bgk_free.
 *
 * Errors.  Every call returns a status code (BGK_OK = 0).  No exception or
 * abort crosses the ABI.  bgk_last_error(ctx) describes the last failure on
 * that context; bgk_last_error(NULL) describes the last failed bgk_init or
 * bgk_step_noalloc of the calling thread.
 */
#ifndef BGK_H
#define BGK_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define BGK_OK 0
#define BGK_E_INVALID 1     /* bad argument (NULL, size, kind, non-positive parameter) */
#define BGK_E_CFL 2         /* Courant sum above 2/3: positivity not guaranteed */
#define BGK_E_UNSUPPORTED 3 /* valid but outside what the library handles */
#define BGK_E_HIP 4         /* a HIP runtime call failed */
#define BGK_E_NONFINITE 5   /* bgk_check: a moment is NaN or infinite */
#define BGK_E_NEGATIVE 6    /* bgk_check: a density or temperature is <= 0 */
#define BGK_E_ALIAS 7       /* input and output buffers are the same */

/* Problem kinds. */
#define BGK_SHOCK_1D 0      /* Sec. 4.1: far-field Maxwellians of Eq. (bc_shock) at both ends */
#define BGK_CAVITY_2D 1     /* Sec. 5.1: four diffuse walls of Eq. (bc_cavity), moving lid on top */
#define BGK_PERIODIC_1D 2   /* periodic test box */
#define BGK_PERIODIC_2D 3   /* periodic test box */
#define BGK_CAVITY_3D 4     /* lid-driven cube: six diffuse walls of Eq. (bc_cavity) (walls 4, 5 across z),
                               the lid at y = y1 moving along x */
#define BGK_PERIODIC_3D 5   /* periodic test box */

#define BGK_STRANG 0        /* R_{dt/2} S_dt R_{dt/2} */
#define BGK_LIE 1           /* R_dt S_dt (Sec. 2.1) */
#define BGK_MINMOD 0        /* second-order minmod-limited upwind */
#define BGK_NOLIMIT 1       /* first-order upwind, Eq. (upwind) */
#define BGK_SHIFT 2         /* translation form of Sec. 2.1: shift by the integer part of the
                               Courant number, Eq. (upwind) over the fraction; one-dimensional
                               kinds, any Courant number (no Courant limit) */

#define BGK_POINT 0         /* relaxation towards the point values of Eq. (Maxw) at the cell's
                               moments (n, V, T) */
#define BGK_CONSERVATIVE 1  /* relaxation towards Eq. (Maxw) at the effective (n~, V~, T~) whose
                               grid moments are exactly the cell's (n, V, T) (Sec. 2.1, the
                               remark on conservation after Eq. (exact)): mass, momentum and
                               energy are conserved by every relaxation on the velocity grid;
                               the collision frequency keeps the cell's own n and T; far-field
                               and wall Maxwellians stay point values */

#define BGK_FP64 0          /* f stored and streamed in double */
#define BGK_FP32 1          /* f stored and streamed in float; moments, Maxwellian
                               parameters and all reductions in double; each stored
                               value is computed in double and rounded to float
                               stochastically (unbiased), see bgk_set_rounding_seed */

/* One problem instance (Sec. 2.1 grid, Sec. 4.1 / 5.1 boundary data). */
typedef struct bgk_problem {
    int kind;               /* BGK_SHOCK_1D, BGK_CAVITY_2D, BGK_PERIODIC_1D/2D, BGK_CAVITY_3D, BGK_PERIODIC_3D */
    int nx, ny;             /* spatial cells (ny ignored for 1D kinds) */
    double x0, x1, y0, y1;  /* spatial box */
    int nv[3];              /* velocity cells per component (even, 2..128) */
    double vlo[3], vhi[3];  /* velocity box; nodes at cell centres */
    double kn;              /* Knudsen number, > 0 */
    double omega;           /* viscosity exponent: nu = n T^(1-omega) / Kn */
    double cfl;             /* used when dt <= 0: dt = cfl / max_j sum_d |v_d|/dx_d */
    double dt;              /* > 0: time step as given */
    double mach;            /* shock: upstream Mach number (Eq. RH), > 1 */
    double lid_mach;        /* cavity: lid speed as a Mach number at T_r, U_W = Ma sqrt(5/6) */
    double t_wall;          /* cavity: wall temperature, > 0 */
    int splitting;          /* BGK_STRANG or BGK_LIE */
    int limiter;            /* BGK_MINMOD, BGK_NOLIMIT or BGK_SHIFT (all instances of a context
                               use BGK_SHIFT or none does) */
    int maxwellian;         /* BGK_POINT or BGK_CONSERVATIVE (per instance) */
    int reduced;            /* 1: reduced velocity space (the projection the paper cites in
                               Sec. 3 and Sec. 6): the components the problem does not stream
                               along are integrated out.  Two-dimensional kinds: nv[2] = 2,
                               plane jz = 0 of f holds g = int f dv_z and plane 1
                               h = int v_z^2 f dv_z on the (v_x, v_y) grid.  One-dimensional
                               kinds: nv[1] = 1, nv[2] = 2, g = int f dv_y dv_z and
                               h = int (v_y^2 + v_z^2) f dv_y dv_z on the v_x grid.  V = 0 along
                               the components out and the integrals of Eq. (Maxw) are exact;
                               their vlo, vhi are ignored; the minmod limiter acts on g and h
                               separately.  0: full velocity space.  The same for all instances
                               of a context.  No reverse sweep.  Not for 3D kinds. */
    int nz;                 /* 3D kinds: spatial cells along z (ignored otherwise).  The v_z nodes
                               must change sign between two planes jz - 1, jz with jz even (an even
                               count of nodes on either side: nv[2] divisible by 4 on a box
                               symmetric about 0), else BGK_E_UNSUPPORTED */
    double z0, z1;          /* 3D kinds: spatial box along z */
} bgk_problem;

typedef struct bgk_ctx bgk_ctx;

/* Create a context for n_probs instances stepped together (one launch per
 * kernel for all of them).  All instances must share the velocity grid;
 * their dimensions may differ (a shock batched with cavities): the kernels
 * run at the highest dimension of the batch, and an instance streams along
 * its own directions only, with the same values as alone (contexts in the
 * reduced velocity space, whose layout depends on the dimension, hold one
 * dimension only; mixed contexts have no reverse sweep).  Validates every field, computes each
 * instance's dt, and allocates the context's small device data (per-cell
 * table entries and moment partial sums, no f-sized buffer) on the current
 * device.  precision: BGK_FP64 or BGK_FP32.
 * Errors: BGK_E_INVALID (also for a maxwellian field other than BGK_POINT and
 * BGK_CONSERVATIVE), BGK_E_CFL (Courant sum > 2/3; not checked for
 * BGK_SHIFT), BGK_E_UNSUPPORTED (also for BGK_SHIFT on a two-dimensional
 * kind or mixed with other limiters in one context, and when one workgroup's
 * table entries, 2 (Nvx + Nvy + Nvz) values per
 * stencil slot, exceed the device's LDS per workgroup), BGK_E_HIP.  On
 * failure *out is NULL. */
int bgk_init(const bgk_problem *probs, int n_probs, int precision, bgk_ctx **out);

/* Release the context and its device memory (synchronises the device). */
int bgk_free(bgk_ctx *ctx);

/* Human-readable description of the last error (never NULL). */
const char *bgk_last_error(const bgk_ctx *ctx);

/* Sizes: total f elements over all instances, total spatial cells, and
 * the bytes of the caller-owned workspaces: ws_step_bytes for bgk_step and
 * bgk_autotune (one f-sized buffer), ws_adjoint_bytes for bgk_step_adjoint
 * (two f-sized buffers and one byte per element of f, rounded up to 256).
 * Any output pointer may be NULL. */
int bgk_sizes(const bgk_ctx *ctx, size_t *f_elems, size_t *n_cells, size_t *ws_step_bytes,
              size_t *ws_adjoint_bytes);

/* Per-instance layout: element offset of the instance in f, index of its
 * first cell in per-cell arrays, and its time step. */
int bgk_instance_info(const bgk_ctx *ctx, int inst, size_t *f_offset, size_t *cell_offset, double *dt);

/* Write the initial state into f (device, f_elems elements): the
 * Rankine-Hugoniot step of Sec. 4.1 for shocks (upstream state for x < 0,
 * downstream for x >= 0), the gas at rest (n = T = 1) otherwise. */
int bgk_initial_state(bgk_ctx *ctx, void *f, void *stream);

/* Advance all instances by n_steps >= 0 time steps:
 * f_out = (one step)^n_steps (f_in).  f_in is read only; f_out must not
 * overlap f_in (BGK_E_ALIAS).  Both hold f_elems elements on the device.
 * ws: the caller's device workspace of ws_step_bytes (bgk_sizes), the
 * ping-pong buffer of the intermediate streaming passes; its contents are
 * overwritten.  It may be NULL for n_steps <= 1 (BGK_E_INVALID for
 * n_steps >= 2) and must not overlap f_in or f_out (BGK_E_ALIAS).  With
 * graph replay on, the workspace address is part of the captured graph. */
int bgk_step(bgk_ctx *ctx, const void *f_in, void *f_out, int n_steps, void *ws, void *stream);

/* Allocation-free variant of bgk_step, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It takes the problems instead of a
 * context and advances them by n_steps exactly as a context made by
 * bgk_init(probs, n_probs, precision, ...) would in its first bgk_step call:
 * same validation and status codes, the default launch shape (no tuned
 * shape), graph replay and kernel timing off, FP32 rounding counters
 * 0 .. n_steps.  f_in, f_out and ws are as for bgk_step (ws of the
 * ws_step_bytes a context would report: the f bytes, the caller's).  It
 * calls no hipMalloc, hipFree or other allocating routine: the device data a
 * context would own (instance tables, Maxwellian table entries, moment
 * partial sums, the rounding counter) lives in one static device array of
 * BGK_NOALLOC_SCRATCH_MIB MiB per GPU, held until the process ends; problems
 * that need more return BGK_E_UNSUPPORTED before any device work.  The
 * array's device address is looked up at the first call on each device.
 * Every call on a GPU shares that GPU's array and leaves its contents there:
 * calls that overlap in time on one GPU (other streams, other threads) race
 * and must be serialised by the caller.  Asynchronous on `stream`; on
 * failure bgk_last_error(NULL) describes the error. */
#define BGK_NOALLOC_SCRATCH_MIB 64
int bgk_step_noalloc(const bgk_problem *probs, int n_probs, int precision, const void *f_in, void *f_out,
                     int n_steps, void *ws, void *stream);

/* Moments of Eq. (macroscopic) of f, per cell: mom[cell][5] =
 * (n, Vx, Vy, Vz, T), double, device, n_cells * 5 elements. */
int bgk_moments(bgk_ctx *ctx, const void *f, double *mom, void *stream);

/* Check f: computes its moments and returns BGK_E_NONFINITE or
 * BGK_E_NEGATIVE if any cell has a non-finite moment or n <= 0 or T <= 0
 * (synchronises the stream). */
int bgk_check(bgk_ctx *ctx, const void *f, void *stream);

/* Launch shape of the streaming kernel (engineering interface; results do
 * not depend on it beyond rounding of the moment sums).  A shape is
 * (vec, unroll, vsplit, persist): jx values per lane task (1, 2 or 4; 4 only
 * for BGK_FP32, and only if it divides Nvx with one v_x sign per group),
 * unroll: the software pipeline of the jz loop (1: one plane per stage, one
 * in flight ahead; 2: two planes per stage, one stage ahead; 3, 4: one plane
 * per stage, 2 or 3 planes ahead), jz chunks per cell (one work item each,
 * 1 .. a context-dependent maximum), and persist: 0 launches one workgroup
 * per work item, k > 0 launches k workgroups per compute unit that walk the
 * items of all instances (one persistent launch for a batch).  Vec is 1
 * for BGK_SHIFT streaming, reduced velocity spaces and 3D kinds; 3D kinds
 * take unroll 1 or 2.  BGK_SHIFT contexts take unroll 1 (the per-cell
 * translation kernel) or, where its row tiles fit, 2 (the row-tile kernel).
 * bgk_init picks a default.  bgk_autotune times every valid shape on the
 * state f (device, f_elems elements, read only; synchronises the stream) and
 * keeps the fastest by the steady time of a real step (streaming pass and
 * table preparation, ((2 + n) steps - 2 steps) / n).  The sweep times n = 8
 * steps per shape after an untimed warm-up of a few steps; the four fastest
 * are then timed twice more with n = 32 after 16 untimed steps and ranked
 * by the better of those two timings alone.  The timed steps write into `scratch` (the
 * caller's device buffer of f_elems elements, overwritten) with `ws` (of
 * ws_step_bytes) as their workspace; f, scratch and ws must not overlap
 * (BGK_E_ALIAS), none may be NULL (BGK_E_INVALID).  On an error the
 * previous shape stays in use; bgk_get_launch reports the shape in use
 * and, after autotuning, the measured time per step in microseconds;
 * bgk_set_launch applies a shape (BGK_E_INVALID if not valid for the
 * context). */
int bgk_autotune(bgk_ctx *ctx, const void *f, void *scratch, void *ws, void *stream);
int bgk_get_launch(const bgk_ctx *ctx, int *vec, int *unroll, int *vsplit, int *persist, double *tuned_us);
int bgk_set_launch(bgk_ctx *ctx, int vec, int unroll, int vsplit, int persist);

/* Graph replay.  When on (default off), bgk_step captures every launch of
 * the call after the one that sets the rounding counter (moments of f_in,
 * tables, all n_steps streaming passes and tables, closing relaxation) into
 * one hipGraph the first time a combination (f_in, f_out, ws, n_steps,
 * timing on or off) is used, and replays that graph when the combination
 * comes again; up to four graphs are kept per context (the least recently
 * used is dropped), until the launch shape changes, graph replay is
 * switched off or the context is freed.  The buffer addresses are part of a
 * graph: do not free and reuse them for other buffers while graph replay is
 * on.  Ignored while kernel timing is on (HIP reports no elapsed time for
 * events that graph nodes record, so timed calls launch eagerly) and on the
 * NULL (legacy default) stream, which cannot be captured. */
int bgk_set_graph(bgk_ctx *ctx, int on);

/* Timing of the streaming kernel.  capacity > 0 turns timing on and creates
 * that many HIP event pairs up front (more are created on demand); while on,
 * bgk_step records a pair around every launch of the streaming kernel on
 * `stream` (calls launch eagerly while timing is on).  capacity = 0 turns
 * timing off.  bgk_timing synchronises and returns the summed device time
 * (ms) and the launch count since the last reset, then resets. */
int bgk_set_timing(bgk_ctx *ctx, int capacity);
int bgk_timing(bgk_ctx *ctx, double *ms, int *launches);

/* Rounding seed of the BGK_FP32 path.  Stored values are rounded up or down
 * to a neighbouring float with probabilities proportional to their distance
 * (unbiased stochastic rounding), because round-to-nearest loses the
 * sub-ulp change per step of a nearly uniform, nearly Maxwellian region and
 * so freezes its slow drift.  The random bits are a hash of (element index
 * within its instance, rounding counter): they do not depend on the launch
 * shape or on batching (results still differ at rounding level between
 * shapes that split a cell's moment sums differently).  The 16 random bits
 * of an element sit at the top of the 29 bits a float drops from a double,
 * so the rounding is unbiased to within 2^-16 ulp.  A call bgk_step(..., n, ...) uses counters
 * seed .. seed + n - 1 for its streaming passes and seed + n for its closing
 * relaxation, then advances the context's seed by n; bgk_set_rounding_seed
 * sets it (0 after bgk_init) so that a run can be repeated bit for bit.
 * No effect on BGK_FP64. */
int bgk_set_rounding_seed(bgk_ctx *ctx, unsigned int seed);
int bgk_get_rounding_seed(const bgk_ctx *ctx, unsigned int *seed);

/* Reverse sweep of one time step (the discrete adjoint of the step defined
 * above: Sec. 2.1 splitting, Eq. (relaxation) with the moments of
 * Eq. (macroscopic) differentiated through Eq. (Maxw) and Eq. (frequency),
 * the minmod flux-form streaming with the diffuse-wall re-emission of
 * Eq. (bc_cavity), whose wall density makes the net wall mass flux zero).
 *   lam_n = (d step / d f)^T lam_next   evaluated at f_n,
 *   grad_params[2k]   += sum lam_next . d step / d Kn     (instance k),
 *   grad_params[2k+1] += sum lam_next . d step / d T_w    (instance k; 0 for
 *                                                           non-cavity kinds).
 * The inner product is the plain element sum over f's layout (no dV weight).
 * f_n, lam_next and lam_n are device arrays of f_elems elements in the
 * context's precision (FP32: f and the adjoint stored in float, every
 * moment, table and reduction in double); lam_n must not alias either input
 * (BGK_E_ALIAS).  grad_params is a device array of 2 * n_probs doubles that
 * the call ACCUMULATES into (zero it before the first step of a sweep).
 * Minmod branch decisions are those of the forward map at f_n: a limited
 * slope is differentiated as 0 unless both differences have the same strict
 * sign, else as the smaller-magnitude difference (the backward one on a tie
 * of magnitudes); the call's own recomputation of the forward streaming
 * pass records them.  ws: the caller's device workspace of ws_adjoint_bytes
 * (bgk_sizes; two f-sized intermediate states and the branch record,
 * overwritten), not overlapping f_n, lam_next or lam_n (BGK_E_ALIAS); NULL
 * gives BGK_E_INVALID.  The first call allocates the context's per-cell
 * reverse-sweep coefficients; BGK_E_HIP if that fails, BGK_E_UNSUPPORTED for
 * BGK_SHIFT contexts (no reverse sweep of the translation form), for contexts
 * with a BGK_CONSERVATIVE instance (no reverse sweep of the effective
 * parameters' solve) and for 3D kinds.  Asynchronous on `stream`. */
int bgk_step_adjoint(bgk_ctx *ctx, const void *f_n, const void *lam_next, void *lam_n, double *grad_params,
                     void *ws, void *stream);

/* Step records: a forward step that keeps what its reverse step needs, so
 * that the reverse step recomputes nothing (the adjoint of one step of
 * Eq. (relaxation) and the streaming of Sec. 2.1, as bgk_step_adjoint).
 * A record holds h = S(R_a f_n) as the step stored it, the per-cell totals
 * of the FP64 moment sums of f_n and of h, and the minmod branch of every
 * limited slope the streaming pass evaluated (one byte per element); its
 * size, bgk_record_bytes, is about one f plus a quarter (FP32) or an
 * eighth (FP64) of one, and a record stays valid for any later launch
 * shape of the context.
 *
 * bgk_step_record: f_out = one step of f_in (as bgk_step with n_steps = 1:
 * the same rounding counter use and the same trajectory up to the rounding
 * of the moment sums, whose order can follow the launch shape), and the
 * step's record into rec (device, bgk_record_bytes, overwritten).  f_in,
 * f_out and rec must not overlap (BGK_E_ALIAS); NULL gives BGK_E_INVALID;
 * BGK_E_UNSUPPORTED for the contexts bgk_step_adjoint rejects.
 *
 * bgk_step_adjoint_record: the reverse step of bgk_step_adjoint at f_n,
 * reading the record rec that bgk_step_record wrote for the step from f_n
 * instead of recomputing it; same outputs, accumulation of grad_params and
 * errors.  ws: the caller's workspace of ws_adjoint_bytes, of which the
 * first f-sized part is used; ws and lam_n must not overlap f_n, rec,
 * lam_next or each other (BGK_E_ALIAS).  Asynchronous on `stream`. */
/* bgk_adjoint_sweep_record: the reverse sweep of n >= 0 recorded steps in
 * one call: lambda^0 = J_0^T ... J_{n-1}^T lambda^n, with f[i] the state at
 * the start of step i and rec[i] its record (host arrays of n device
 * pointers, i = 0 .. n-1), lam_N = lambda^n, lam_0 the output; grad_params
 * accumulates every step's parameter gradients, as n calls of
 * bgk_step_adjoint_record would (same lambda^0; the gradient sums in another
 * order).  Steps run from the last to the first, and each step's closing
 * pass also forms the sums at h of the step before it, so the sweep reads
 * lambda one time fewer per step.  ws: ws_adjoint_bytes, of which the first
 * two f-sized parts are used; lam_0 and ws must not overlap lam_N, a state,
 * a record or each other (BGK_E_ALIAS).  Errors as bgk_step_adjoint.
 * Asynchronous on `stream`. */
int bgk_adjoint_sweep_record(bgk_ctx *ctx, int n, const void *const *f, const void *const *rec, const void *lam_N,
                             void *lam_0, double *grad_params, void *ws, void *stream);
int bgk_record_bytes(const bgk_ctx *ctx, size_t *bytes);
int bgk_step_record(bgk_ctx *ctx, const void *f_in, void *f_out, void *rec, void *stream);
int bgk_step_adjoint_record(bgk_ctx *ctx, const void *f_n, const void *rec, const void *lam_next, void *lam_n,
                            double *grad_params, void *ws, void *stream);

/* Shear stress on the moving lid (Sec. 5.1 cavity; the xy momentum flux
 * through the top wall, integrated along it):
 *   L_k = dx * dV * sum_{top cells} [ sum_{v_y>0} v_x v_y f
 *                                     + n_W sum_{v_y<0} v_x v_y Phi_W ],
 * with Phi_W the unit-density wall Maxwellian at (U_W, 0, 0) and T_w and n_W
 * the per-cell wall density that balances the incident flux
 * sum_{v_y>0} v_y f.  Written to L[k] (device, n_probs doubles); 0 for
 * non-cavity instances.  f: device, f_elems elements.  BGK_E_UNSUPPORTED
 * for 3D kinds (as is the gradient below). */
int bgk_lid_shear(bgk_ctx *ctx, const void *f, double *L, void *stream);

/* Gradient of bgk_lid_shear: lam = dL/df (device, f_elems elements in the
 * context's precision, overwritten, zero outside the top row of each
 * cavity; must not alias f) and grad_params[2k+1] += dL_k/dT_w
 * (grad_params[2k] unchanged: L has no explicit Kn dependence). */
int bgk_lid_shear_grad(bgk_ctx *ctx, const void *f, void *lam, double *grad_params, void *stream);

/* Steady-cavity metrics compared in the Table of Sec. 5.2, per instance:
 * out[2k] = D, the mean shear stress on the lid in units of p0 U_W
 * (p0 = 1/2, the pressure of the gas at rest with n = T = 1):
 * D = -L / (p0 U_W (x1 - x0)), L as in bgk_lid_shear; out[2k + 1] = G, the
 * flow rate of the main vortex as Sec. 5.2 defines it: the integral of
 * V_x / U_W along the vertical line through the middle of the cavity (the
 * middle column, or the mean of the two middle columns), from the first
 * zero below the lid (the vortex centre; linear between cell centres) up to
 * the lid (linear extrapolation over the top half cell), or from the bottom
 * wall if there is no zero, divided by the height (y1 - y0).  NaN for
 * non-cavity instances (3D kinds included) and for a lid at rest.  f: device, f_elems elements; out: host, 2 n_probs doubles.
 * Synchronises `stream`; errors: BGK_E_INVALID, BGK_E_HIP. */
int bgk_cavity_metrics(bgk_ctx *ctx, const void *f, double *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* BGK_H */
