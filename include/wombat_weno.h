/*
 * wombat_weno.h -- C ABI of the MI355X (gfx950) WENO5 ideal-MHD stage library.
 *
 * The library advances the eight conserved ideal-MHD variables with the
 * fifth-order characteristic WENO finite-difference scheme of Donnert et al.,
 * "Towards Exascale Simulations of the ICM Dynamo with WENO-Wombat"
 * (arXiv:1808.10633), Sec. 2.1:
 *   - per sweep direction, the interface flux of each characteristic field by
 *     eq. (1), with the WENO5 interpolant of eq. (2), the nonlinear weights of
 *     eqs. (3)-(4) (epsilon = 1e-6) and the smoothness indicators of
 *     eqs. (5)-(7), after a Roe-type decoupling of the 8 PDEs and a
 *     Lax-Friedrichs flux splitting;
 *   - flux differences in x, y and z (Sec. 2.2: unsplit sweeps, one final
 *     update), constrained transport of B on a staggered mesh (Sec. 2.1),
 *   - a four-stage, fourth-order Runge-Kutta integrator (Sec. 2.1),
 *   - 3 ghost zones per side (Sec. 2.2).
 * The paper leaves the eigenvectors, the interface mean state, the CT edge
 * average and the time-step rule to unpublished work; this library uses:
 * the arithmetic mean of the primitive variables of the two cells, the
 * seven-wave eigenvectors with the Roe-Balsara normalisation (normal field
 * held fixed, zero normal-field flux), the local per-field Lax-Friedrichs
 * speed max|lambda^s| over the six stencil cells, the four-face mean of the
 * transverse-field fluxes as edge EMF with the cell field advanced by the
 * mean of its two face updates, classical RK4, and
 * dt = C / max_cells sum_d (|v_d| + c_f,d)/dx_d.  Units: Heaviside-Lorentz
 * (magnetic pressure B^2/2), ideal-gas equation of state.
 *
 * STATE LAYOUT (every state argument):
 *   caller-owned device memory, contiguous, u[v][k][j][i] with i fastest;
 *   v = 0..7 = (rho, rho vx, rho vy, rho vz, Bx, By, Bz, E);
 *   dims (nx+2gx) x (ny+2gy) x (nz+2gz), g = 3 on an axis with n > 1 and
 *   g = 0 on an inactive axis (n = 1); point values at cell centres.
 *   Element type: double for WW_FP64, float for WW_FP32_MIXED.
 *   A 256-byte aligned base is recommended, 8-byte alignment is required.
 *
 * ERRORS: every call returns WW_OK (0) or a negative ww_status.  Invalid
 * arguments are reported before any device work and leave no side effect.
 * A HIP failure makes the context's error sticky: later calls return
 * WW_ERR_HIP until wombat_weno_destroy.  No C++ exception crosses the ABI.
 * wombat_weno_last_error(ctx) gives a message for the last failure
 * (wombat_weno_last_error(NULL) for failures of wombat_weno_init).
 *
 * THREADING AND ORDERING: a context is used by one host thread at a time;
 * several contexts may coexist.  All device work of a context is enqueued on
 * the stream given in the configuration (0 = the null stream), in call
 * order.  Calls documented as synchronous wait for that stream.  The library
 * allocates device memory only in wombat_weno_init / wombat_weno_batch_init
 * and frees it only in the matching destroy call; it never frees caller
 * memory.  No other call allocates device or pinned host memory (stages,
 * steps, routing, autotuning and graph replay included), so stages can be
 * captured in HIP graphs; wombat_weno_alloc_count() lets a caller check this.
 */
#ifndef WOMBAT_WENO_H
#define WOMBAT_WENO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WOMBAT_WENO_ABI_VERSION 6

typedef enum {
    WW_OK = 0,
    WW_ERR_INVALID_ARG = -1,  /* bad pointer, size, alias or configuration   */
    WW_ERR_UNSUPPORTED = -2,  /* valid request the library does not provide */
    WW_ERR_OOM = -3,          /* device allocation failed in init            */
    WW_ERR_HIP = -4,          /* a HIP runtime call failed (sticky)          */
    WW_ERR_NONPHYSICAL = -5,  /* rho <= 0, p <= 0 or a non-finite value      */
    WW_ERR_USER_BC = -6,      /* a user boundary callback returned non-zero  */
    WW_ERR_STATE = -7         /* call not allowed in the context's state     */
} ww_status;

typedef enum { WW_FP64 = 0, WW_FP32_MIXED = 1 } ww_precision;
/* Nonlinear weights of the interpolant.  WW_WEIGHTS_JS: eq. (3)-(5), the
 * paper's choice (Sec. 2.1).  WW_WEIGHTS_Z: the WENO-Z weights of Borges et
 * al. (2008) with exponent 1, alpha_k = d_k (1 + tau5 / (eps + IS_k)),
 * tau5 = |IS_0 - IS_2|, same smoothness indicators, linear weights and eps;
 * offered for the comparison the paper argues (JS is the more robust of the
 * two at shocks), on the single-grid operator only. */
typedef enum { WW_WEIGHTS_JS = 0, WW_WEIGHTS_Z = 1 } ww_weights;
/* Time integrator of wombat_weno_step.  WW_RK4: the classical four-stage,
 * fourth-order Runge-Kutta of Sec. 2.1 (low-storage form).  WW_SSPRK3: the
 * three-stage, third-order strong-stability-preserving scheme of Shu &
 * Osher (1988), u1 = u + dt L(u), u2 = 3/4 u + 1/4 (u1 + dt L(u1)),
 * u^{n+1} = 1/3 u + 2/3 (u2 + dt L(u2)); an ablation of the paper's
 * choice, single-grid operator and wombat_weno_step only. */
typedef enum { WW_RK4 = 0, WW_SSPRK3 = 1 } ww_integrator;
/* Lax-Friedrichs speed alpha^s of eq. (1).  WW_LF_LOCAL: per interface, the
 * largest |lambda^s| of field s over its six stencil cells (the reading of
 * the paper's "simple Lax-Friedrichs splitting" used throughout).
 * WW_LF_GLOBAL: per sweep direction and stage, the largest |lambda^s| over
 * every cell the sweep reads (one extra FP64 reduction pass per direction
 * and stage); an ablation, single-grid operator only. */
typedef enum { WW_LF_LOCAL = 0, WW_LF_GLOBAL = 1 } ww_lf_speed;
typedef enum { WW_BC_PERIODIC = 0, WW_BC_OUTFLOW = 1, WW_BC_USER = 2 } ww_bc;
/* Storage of B.  WW_B_CELL: cell-centred B; constrained transport advances
 * each staggered face by -(curl E).n and the cell field by the mean of its
 * two faces (the reading used throughout; invariant: the corner divergence).
 * WW_B_FACE: staggered storage, the mesh of Ryu et al. (1998) that Sec. 2.1
 * names: the B_d slot of a cell holds the normal field of its lower d-face
 * (at i - 1/2 along d); the sweeps see the mean of a cell's two faces; each
 * face advances by -(curl E).n from the same edge EMFs (invariant: the face
 * divergence); an ablation, periodic boxes, single-grid operator only.  With
 * B_cell = mean of the faces the two forms give the same cell field up to
 * round-off. */
typedef enum { WW_B_CELL = 0, WW_B_FACE = 1 } ww_b_storage;

/* User boundary hook: called for each WW_BC_USER face (0..5 = -x,+x,-y,+y,
 * -z,+z) whenever ghosts are filled, after the built-in faces of the same
 * axis.  It must enqueue its device work on `stream` (a hipStream_t) and fill
 * the 3-deep ghost slab of that face for all 8 variables; return 0 on
 * success. */
typedef int (*ww_user_bc_fn)(void *user, void *d_u, int face, void *stream);

typedef struct {
    int nx, ny, nz;          /* interior cells, >= 1; 1 marks an inactive axis;
                                an active axis needs n >= 3                    */
    int ng;                  /* ghost cells per side on active axes: must be 3 */
    double dx, dy, dz;       /* cell widths, > 0                               */
    double gamma;            /* ratio of specific heats, > 1                   */
    double cfl;              /* Courant number in (0, 1]                       */
    double eps;              /* WENO epsilon of eq. (4), > 0 (paper: 1e-6)     */
    int precision;           /* ww_precision                                   */
    int bc[6];               /* ww_bc per face -x,+x,-y,+y,-z,+z; periodic
                                must be set on both faces of an axis           */
    ww_user_bc_fn user_bc;   /* required if any face is WW_BC_USER             */
    void *user_bc_ctx;       /* passed back to user_bc                         */
    void *stream;            /* hipStream_t for all work; NULL = null stream   */
    int device;              /* HIP device ordinal                             */
    int weights;             /* ww_weights (added in ABI 2); the batched and
                                learned forms accept WW_WEIGHTS_JS only        */
    int integrator;          /* ww_integrator (added in ABI 3); the batched
                                and learned forms and wombat_weno_stage accept
                                WW_RK4 only                                   */
    int lf_speed;            /* ww_lf_speed (added in ABI 4); the batched and
                                learned forms accept WW_LF_LOCAL only          */
    int learned;             /* 1: wombat_weno_init also allocates the learned
                                router's buffers (see wombat_weno_set_router);
                                FP32, WW_WEIGHTS_JS, WW_RK4 and WW_LF_LOCAL
                                only; 0 (default): no routing (added in ABI 5) */
    int slab_planes;         /* 0 (default): stages work on the whole box.
                                >= 3: stages run in z-slabs of this many planes
                                (needs nz >= 3; WW_RK4, WW_LF_LOCAL, no router):
                                face fluxes are stored for one slab, not the
                                box, wombat_weno_step keeps two work arrays
                                instead of three, and wombat_weno_stage may
                                write its output over its input (added in ABI 5).
                                Results are identical bit for bit.           */
    int b_storage;           /* ww_b_storage (added in ABI 6); WW_B_FACE needs
                                periodic faces and no slab_planes or router  */
} wombat_weno_config;

typedef struct wombat_weno wombat_weno_t;

/* ABI version of the loaded library (WOMBAT_WENO_ABI_VERSION). */
int wombat_weno_abi_version(void);

/* Fill *cfg with defaults: 32^3 unit box, ng 3, gamma 5/3, cfl 0.4,
 * eps 1e-6, WW_FP64, all faces periodic, null stream, device 0,
 * WW_WEIGHTS_JS, WW_RK4, WW_LF_LOCAL, learned 0, slab_planes 0, WW_B_CELL.
 * Returns WW_ERR_INVALID_ARG if cfg is NULL. */
int wombat_weno_config_default(wombat_weno_config *cfg);

/* Check a configuration without touching any device.  WW_OK or
 * WW_ERR_INVALID_ARG (message in wombat_weno_last_error(NULL)). */
int wombat_weno_validate_config(const wombat_weno_config *cfg);

/* Number of elements (not bytes) of one padded state array. */
int64_t wombat_weno_state_elems(const wombat_weno_config *cfg);

/* Create a context: validates cfg, selects cfg->device and allocates every
 * device buffer the context will use: three state-sized work arrays (two
 * with slab_planes), the face fluxes of the three sweeps (of one slab with
 * slab_planes, plus a delay buffer of three planes), small reduction
 * buffers, with
 * WW_LF_GLOBAL 57 KB of LF-speed partials, and with cfg->learned the
 * learned form's buffers (a state-sized backup, the packed parameters, a
 * queue of one 8-byte entry per face of the largest sweep, one decision
 * byte per face of every sweep).  *out is written only on success.
 * Errors: WW_ERR_INVALID_ARG, WW_ERR_OOM, WW_ERR_HIP, WW_ERR_UNSUPPORTED
 * (cfg->learned with a precision or scheme the router does not serve;
 * slab_planes with WW_SSPRK3, WW_LF_GLOBAL or learned; WW_B_FACE with a
 * non-periodic face, slab_planes or learned).  WW_B_FACE adds one
 * state-sized work array (the cell-centred state the sweeps read). */
int wombat_weno_init(const wombat_weno_config *cfg, wombat_weno_t **out);

/* Release a context and its device memory.  NULL is allowed. */
void wombat_weno_destroy(wombat_weno_t *ctx);

/* Message of the last failure on ctx (NULL: of the last failed init or
 * validation on this thread).  The string is owned by the library. */
const char *wombat_weno_last_error(const wombat_weno_t *ctx);

/* Fill the 3-deep ghost zones of d_u (periodic copy, zero-gradient outflow
 * or the user hook), axis by axis (Sec. 2.2).  Asynchronous. */
int wombat_weno_fill_ghosts(wombat_weno_t *ctx, void *d_u);

/* CFL time step dt = cfl / max over interior cells of
 * sum_d (|v_d| + c_f,d)/dx_d, reduced in FP64 on the device (with
 * WW_B_FACE, of the cell-centred state); waits for the stream and writes
 * *dt.  WW_ERR_NONPHYSICAL if any interior cell has
 * rho <= 0, p <= 0 or a non-finite value (then *dt is not written). */
int wombat_weno_cfl_dt(wombat_weno_t *ctx, const void *d_u, double *dt);

/* As wombat_weno_cfl_dt but asynchronous: writes dt (double) to device
 * memory d_dt and, to d_flag (int32, device), 0 or the number of
 * non-physical cells (dt is then not meaningful). */
int wombat_weno_cfl_dt_device(wombat_weno_t *ctx, const void *d_u, double *d_dt,
                              int32_t *d_flag);

/* Semi-discrete right-hand side L(U) of Sec. 2.1: fills the ghosts of d_u,
 * runs the x, y, z characteristic WENO sweeps, differences the fluxes of
 * rho, m, E and advances B by constrained transport; writes L(U) into the
 * interior of d_dudt (ghosts of d_dudt untouched).  d_dudt must not alias
 * d_u.  Asynchronous. */
int wombat_weno_rhs(wombat_weno_t *ctx, void *d_u, void *d_dudt);

/* One Runge-Kutta stage s in {0,1,2,3} of the classical RK4 step of size dt
 * (Sec. 2.1), in the low-storage form
 *   s=0: acc = u0 + dt/6 L(u0),   out = u0 + dt/2 L(u0)   (pass us_in == u0)
 *   s=1: acc += dt/3 L(us),       out = u0 + dt/2 L(us)
 *   s=2: acc += dt/3 L(us),       out = u0 + dt   L(us)
 *   s=3:                          out = acc + dt/6 L(us)   (u0 unused)
 * Ghosts of d_us_in are filled first; interior cells of d_acc and d_us_out
 * are written.  d_us_out may alias d_u0 (pointwise), but not d_acc, nor
 * d_us_in unless the context has slab_planes (then the stage writes over its
 * input: the last three output planes of each slab wait in a delay buffer
 * until the next slab has read its input, and the ghost cells of those
 * planes are left zero; ghosts are refilled before every read).  dt must be
 * finite and > 0.  Asynchronous.  WW_ERR_UNSUPPORTED on a context
 * configured with WW_SSPRK3. */
int wombat_weno_stage(wombat_weno_t *ctx, int s, double dt, const void *d_u0,
                      void *d_us_in, void *d_acc, void *d_us_out);

/* A full step of d_u in place using the context's work arrays: the four
 * RK4 stages above, or the three SSP-RK3 stages with WW_SSPRK3.
 * dt <= 0 computes the CFL step first (synchronous; may return
 * WW_ERR_NONPHYSICAL).  *dt_used (may be NULL) receives the step taken.
 * Asynchronous when dt > 0. */
int wombat_weno_step(wombat_weno_t *ctx, void *d_u, double dt, double *dt_used);

/* FP64 sums of the 8 conserved variables over the interior cells (fixed
 * reduction order, deterministic).  Synchronous. */
int wombat_weno_sums(wombat_weno_t *ctx, const void *d_u, double out[8]);

/* Corner divergence of the cell-centred field: for each corner i+1/2 (and
 * j+1/2, k+1/2 on active axes), i = 0..n-1, the sum over active axes d of the
 * mean over the adjacent cell pairs of (B_d(+1) - B_d(0))/dx_d.  Fills the
 * ghosts of d_u first.  Writes max |div B| and its mean.  With WW_B_FACE:
 * the face divergence sum_d (b_d(i+1/2) - b_d(i-1/2))/dx_d of every cell
 * instead.  Synchronous. */
int wombat_weno_divb(wombat_weno_t *ctx, void *d_u, double *max_abs, double *l1);

/* Kernel timing: average device time in milliseconds per launch of each
 * kernel of a step on the state d_u, measured with HIP events recorded on
 * the context's stream around `reps` back-to-back launches after one untimed
 * launch (reps in 1..1000): ms[0] the ghost fill of all axes, ms[1..3] the
 * x, y and z sweeps (0 for an inactive axis), ms[4] the flux-difference/CT/
 * update kernel in the stage forms a step runs (the mean over the four RK4
 * stages, or the three SSP-RK3 stages, with u0 = d_u and the context's work
 * arrays as accumulator and output, dt = 0), ms[5] the CFL reduction (both
 * passes), ms[6] the update writing L(U) only (the form of wombat_weno_rhs).
 * A step costs about ms[5] + stages * (ms[0] + ms[1] + ms[2] + ms[3] + ms[4]).
 * With slab_planes, ms[1..4] and ms[6] are the launches of all slabs of a
 * stage.
 * d_u's ghosts are filled; the work arrays are overwritten.  Synchronous. */
int wombat_weno_time_kernels(wombat_weno_t *ctx, void *d_u, int reps, double ms[7]);

/* Device and pinned-host allocations the library has made since it was
 * loaded (all contexts and batches of the process); a diagnostic that
 * shows that calls after init allocate nothing. */
int64_t wombat_weno_alloc_count(void);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * right-hand side of wombat_weno_rhs without a context.  cfg is validated as
 * in wombat_weno_init (cfg->learned must be 0; the stream and device of cfg
 * are used); d_u (its ghosts are filled) and d_dudt (interior written) are
 * caller-owned device states of cfg's layout and precision, d_dudt must not
 * alias d_u.  The face fluxes of the three sweeps (and, with WW_LF_GLOBAL,
 * 57 KB of partial maxima) are kept in one fixed 64 MiB device array of the
 * library, 256-byte aligned per buffer: boxes whose face fluxes exceed it
 * (e.g. beyond ~70^3 in FP64 or ~90^3 in FP32) get WW_ERR_INVALID_ARG and a
 * message.  The call allocates nothing (no hipMalloc, no pinned memory,
 * nothing from the caller); each GPU it runs on holds its own copy of the
 * array until the process ends.  Every buffer is written before it is read
 * in a call, so no contents carry over between calls, but all calls on one
 * GPU share the array: calls that overlap in time on one GPU (other streams,
 * other threads) race.  Results equal wombat_weno_rhs's bit for bit.
 * Asynchronous on cfg->stream.  Errors: WW_ERR_INVALID_ARG, WW_ERR_UNSUPPORTED,
 * WW_ERR_USER_BC, WW_ERR_HIP (message in wombat_weno_last_error(NULL)). */
int wombat_weno_rhs_noalloc(const wombat_weno_config *cfg, void *d_u, void *d_dudt);

/* ------------------------------------------------------------------------
 * Batched form: many independent periodic patches (Sec. 2.2: the domain is
 * cut into patches with their own ghost zones that are computed
 * independently), advanced together by one persistent launch per RK stage.
 *
 * ARENA LAYOUT: one caller-owned device array holds every patch's padded
 * state u[v][k][j][i] (each axis n+6 long, all axes active) starting at the
 * element offset wombat_weno_batch_patch_offset(b, p); total length
 * wombat_weno_batch_arena_elems(b) elements of the configured precision.
 * Every patch is periodic on all faces and has its own CFL time step,
 * computed on the device in stage 0 of every step and kept there.
 * ------------------------------------------------------------------------ */
typedef struct wombat_weno_batch wombat_weno_batch_t;

/* Create a batch of npatch patches; dims (host) holds npatch x (nx, ny, nz),
 * each edge 4..1024 cells (the 3-deep periodic ghosts need at least 3).  From cfg only dx (the cell width of every
 * patch and axis), gamma, cfl, eps, precision, stream and device are used.
 * Allocates three work arenas, the face-flux scratch of up to 4 blocks per
 * CU, the patch table and the patch order (largest first; in each stage the
 * resident blocks take the next patch of that order from a shared counter
 * until none is left).  *out is written only on success.
 * Errors: WW_ERR_INVALID_ARG, WW_ERR_OOM, WW_ERR_HIP, WW_ERR_UNSUPPORTED. */
int wombat_weno_batch_init(const wombat_weno_config *cfg, int npatch, const int32_t *dims,
                           wombat_weno_batch_t **out);

/* Release a batch (NULL allowed). */
void wombat_weno_batch_destroy(wombat_weno_batch_t *b);

/* Message of the last failure on b (NULL: of the last failed batch init). */
const char *wombat_weno_batch_last_error(const wombat_weno_batch_t *b);

/* Elements of one arena; element offset of patch p's padded state (-1 on a
 * bad argument). */
int64_t wombat_weno_batch_arena_elems(const wombat_weno_batch_t *b);
int64_t wombat_weno_batch_patch_offset(const wombat_weno_batch_t *b, int p);

/* One classical RK4 step of every patch of d_arena in place, each with its
 * own CFL time step: four launches of the persistent stage kernel on the
 * configured stream.  Asynchronous.  The arena's ghost zones are neither read
 * nor written: the sweeps take each ghost cell from its periodic image. */
int wombat_weno_batch_step(wombat_weno_batch_t *b, void *d_arena);

/* As nsteps calls of wombat_weno_batch_step, replaying a HIP graph of one
 * step (captured on first use for this arena pointer, recaptured when the
 * pointer or the launch shape changes).  Asynchronous. */
int wombat_weno_batch_graph_steps(wombat_weno_batch_t *b, void *d_arena, int nsteps);

/* Per-patch time step of the last step and count of non-physical cells
 * (0 = healthy; a patch with a non-physical cell gets dt = 0 and is left
 * unadvanced by the step).  Host arrays
 * of npatch entries, either may be NULL.  Synchronous. */
int wombat_weno_batch_dt(wombat_weno_batch_t *b, double *h_dt, int32_t *h_flag);

/* Launch shape in use: faces per y/z sweep tile (4, 8, 12 or 16), blocks per CU,
 * total persistent blocks. */
int wombat_weno_batch_shape(const wombat_weno_batch_t *b, int *ft, int *blocks_per_cu,
                            int *nblocks);

/* Autotuner: if cache_path (a text file, one JSON object per line; may be
 * NULL) holds an entry for this patch set, precision and architecture, use
 * it; otherwise time every launch shape (faces per tile 4, 8, 12 or 16 x
 * 1..4 blocks per CU within the occupancy limit) by the median of five
 * launches of the second RK4 stage (its most expensive form), run on a copy
 * of d_arena in the batch's own work arenas with zero RK weights (so the
 * repeated launches do the same work), keep the fastest, append it to
 * cache_path, and return its median stage time in *best_ms (-1 when taken
 * from the cache).  d_arena is not modified; the call allocates nothing.  The per-patch time steps are recomputed from d_arena.
 * Synchronous. */
int wombat_weno_batch_autotune(wombat_weno_batch_t *b, const void *d_arena, const char *cache_path,
                               double *best_ms);

/* ------------------------------------------------------------------------
 * Learned troubled-interface router.  Not part of the paper's method: a
 * small MLP decides per interface whether the characteristic WENO flux of
 * Sec. 2.1 is needed; interfaces it calls smooth get the linear fifth-order
 * component-wise flux (one Lax-Friedrichs speed max(|v_n| + c_f) over the
 * stencil, weights (2,-13,47,27,-3)/60 on F^+ and the mirror on F^-).
 *
 * MLP: 48 -> 32 (ReLU) -> 32 (ReLU) -> 1 (sigmoid).  Inputs: from the six
 * cells i-2..i+3 of the interface, for each of the 8 conserved variables in
 * the sweep frame (rho, m_n, m_t1, m_t2, B_n, B_t1, B_t2, E), six values
 * x[v*6 + j] = 1 + log2m(y_j / S_v + 1e-8) log10(2)/4 with y_0 the largest
 * first difference on the stencil, y_1 the jump across the interface,
 * y_2..y_4 the largest second to fourth and y_5 the fifth difference
 * (absolute values); S_v the stencil scale of the variable (see
 * wombat_weno_router_sample); log2m Mitchell's log2 (exponent plus mantissa
 * fraction of the FP32 value).
 * Parameters: one FP32 device vector of wombat_mlp_param_count() = 2657
 * values: W1 (32x48 row-major [out][in]), b1 (32), W2 (32x32), b2 (32),
 * w3 (32), b3.  Products run in BF16 on MFMA with FP32 accumulation.
 * Training label ("troubled"): the flux excess below exceeds a threshold
 * (1e-3 by default in the Python training code).
 * ------------------------------------------------------------------------ */

/* Route the sweeps of an FP32 context through the router.  d_theta
 * (device FP32, wombat_mlp_param_count() values, read on the context's
 * stream during this call: a copy packed as BF16 MFMA operands is kept, so
 * later changes to d_theta need another call; NULL switches routing off),
 * threshold in (0,1): an interface is troubled when sigmoid(logit) >
 * threshold (NaN counts as troubled).  mode 0 routes: smooth interfaces
 * take the linear flux in the routed sweep, troubled ones are queued and
 * take the full flux in a second pass; +1 sends every interface to the full
 * flux (the plain sweep) and -1 every one to the linear flux (the routed
 * sweep without evaluating the network).  A call with a non-NULL
 * d_theta needs a context created with cfg.learned = 1, whose init
 * allocated the buffers the router uses; it allocates nothing itself
 * (WW_ERR_STATE on a context without them).
 * wombat_weno_step evaluates the network at its first stage and reuses
 * those decisions (one byte per face, kept in the context) for its other
 * three stages; wombat_weno_stage and wombat_weno_rhs evaluate it on every
 * call.  Full WENO is the fallback: wombat_weno_step with mode 0 keeps u^n
 * in the backup array, and if the routed step leaves a non-physical cell it
 * is redone from u^n with full characteristic WENO on every interface
 * (counted in router_stats).  Stages and rhs calls have no fallback.
 * On 3-D boxes whose x rows have at least 86 faces the sweeps run y, z, x
 * and the routed x sweep (with two fix-up passes after its troubled pass)
 * also applies the rho, m, E part of the stage, as the plain route's fused
 * x sweep does; the result is that of the separate update.
 * WW_ERR_UNSUPPORTED on FP64 contexts (and with WW_WEIGHTS_Z, WW_SSPRK3 or
 * WW_LF_GLOBAL), WW_ERR_INVALID_ARG for a threshold or mode out of range,
 * WW_ERR_STATE without cfg.learned. */
int wombat_weno_set_router(wombat_weno_t *ctx, const float *d_theta, double threshold, int mode);

/* Interfaces routed to the linear flux by the three sweeps of the last
 * right-hand side or stage, the number of interfaces swept, and (if
 * fallbacks is not NULL) how many routed steps were redone with full WENO
 * since init.  Synchronous. */
int wombat_weno_router_stats(wombat_weno_t *ctx, int64_t *smooth, int64_t *total, int64_t *fallbacks);

/* Training data: for n interfaces d_where[s] = (dir, i, j, k) (device,
 * int32 x 4; the coordinate along dir is a face index 0..n_dir, the others
 * interior cell indices) of the state d_u (its ghosts are filled first),
 * write (all device FP32, caller-owned, none NULL):
 *   d_X[s*48..]   the 48 features;
 *   d_dev[s]      the largest deviation of any weight of eq. (3) (any
 *                 field, either side of eq. (1)) from (0.1, 0.6, 0.3);
 *   d_excess[s]   the flux excess max_c |Fc_full - Fc_lin| / (a S_c): the
 *                 characteristic flux against the linear flux, with a the
 *                 largest |v_n| + c_f on the stencil and the stencil scales
 *                 S = max rho (mass), max(|m|_1 + rho a) (momenta),
 *                 max |B|_1 + sqrt(max rho) a (fields), max E (energy),
 *                 |.|_1 the sum of absolute components.
 * A position outside the box (dir not an active axis, a face index outside
 * 0..n_dir, a transverse index outside 0..n-1) gets NaN in all three
 * outputs; the others are unaffected.  WW_ERR_INVALID_ARG for NULL
 * pointers or n < 1.  Asynchronous. */
int wombat_weno_router_sample(wombat_weno_t *ctx, void *d_u, const int32_t *d_where, int n,
                              float *d_X, float *d_dev, float *d_excess);

/* Number of MLP parameters (2657). */
int wombat_mlp_param_count(void);

/* Logits of n samples d_X[n][48] into d_logit[n] (device FP32), on stream
 * (hipStream_t, NULL = null stream).  Asynchronous. */
int wombat_mlp_forward(void *stream, const float *d_theta, const float *d_X, int n, float *d_logit);

/* Workspace (in floats) wombat_mlp_grad needs for n samples. */
int64_t wombat_mlp_grad_workspace(int n);

/* Gradient of the mean binary cross-entropy of sigmoid(logit) against
 * targets d_t[n] over the n samples: d_grad[2657] and, if d_loss is not
 * NULL, the loss.  d_work: wombat_mlp_grad_workspace(n) floats.  The sum
 * over samples runs in a fixed order (deterministic).  Asynchronous. */
int wombat_mlp_grad(void *stream, const float *d_theta, const float *d_X, const float *d_t, int n,
                    float *d_work, float *d_grad, float *d_loss);

/* One Adam step (step >= 1 counts from 1) on the FP32 master parameters
 * with moment vectors d_m, d_v (2657 each, zero before the first step).
 * Asynchronous. */
int wombat_mlp_adam(void *stream, float *d_theta, float *d_m, float *d_v, const float *d_grad,
                    int step, float lr, float beta1, float beta2, float eps);

#ifdef __cplusplus
}
#endif
#endif
