/*
 * wcnst.h -- C ABI of the MI355X (gfx950) WCNS-T solver core.
 *
 * WCNS-T ("TCNS") is the weighted compact nonlinear scheme of Zhang, Zhang &
 * Xu, "Towards optimal high-order compact schemes for simulating
 * compressible flows" (arXiv:1810.07806): a fifth-order node-to-midpoint
 * interpolation whose three 3-point candidates are kept or discarded by the
 * TENO-like cut-off of Sec. 2.3 (Eqs. (16)-(19)), an upwind midpoint flux
 * (Sec. 2.2, Eq. (6)), and the explicit midpoint-and-node-to-node difference
 * of Sec. 2.1, Eq. (5), advanced in time with third-order SSP Runge-Kutta
 * (Sec. 2).  For the Euler equations the interpolation acts on
 * characteristic variables (Sec. 3).
 *
 * Conventions for every entry point:
 *   - All state pointers are DEVICE pointers to FP64 arrays laid out
 *     U[v][y][x] (x fastest, contiguous, no padding), v = 0..nvar-1:
 *       advection / Burgers: nvar = 1, (u)
 *       Euler 1D:            nvar = 3, (rho, rho*u, E)
 *       Euler 2D:            nvar = 4, (rho, rho*u, rho*v, E)
 *     They are owned by the caller and must stay valid until the work queued
 *     on the solver's stream has finished.
 *   - The library never allocates device memory.  The caller provides one
 *     device workspace of wcnst_workspace_size() bytes at creation; it must
 *     outlive the handle.
 *   - Work is queued on the HIP stream given at creation and runs
 *     asynchronously unless the entry point says otherwise.
 *   - Every entry point returns a wcnst_status; 0 is success.  Errors found
 *     on the device (non-physical states) are sticky and surface at the next
 *     synchronising call.  wcnst_last_error() gives a thread-local message.
 *   - Handles are not thread-safe; one handle per host thread.
 */
#ifndef WCNST_H
#define WCNST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t wcnst_status;

enum {
    WCNST_OK = 0,
    WCNST_E_INVALID_ARG = 1,  /* bad descriptor, pointer, size or workspace */
    WCNST_E_NONPHYSICAL = 2,  /* rho <= 0, p <= 0 or a non-finite value after a stage */
    WCNST_E_MAX_STEPS = 3,    /* wcnst_solve hit max_steps before t_final */
    WCNST_E_HIP = 4           /* a HIP runtime call failed */
};

enum { WCNST_ADVECTION = 0, WCNST_BURGERS = 1, WCNST_EULER = 2 };
enum { WCNST_PERIODIC = 0, WCNST_ZERO_GRADIENT = 1, WCNST_REFLECT = 2, WCNST_FIXED = 3 };
enum { WCNST_ROE = 0, WCNST_LF = 1, WCNST_VANLEER = 2 };
enum { WCNST_TENO = 0, WCNST_LINEAR = 1, WCNST_JS = 2, WCNST_Z = 3 };
enum { WCNST_MND = 0, WCNST_MD = 1, WCNST_HWCNS = 2 };

/* Problem descriptor.  Initialise with wcnst_desc_init(), then set fields. */
typedef struct wcnst_desc {
    uint32_t struct_size; /* sizeof(wcnst_desc), for ABI versioning */
    int32_t ndim;         /* 1 or 2 (2D requires WCNST_EULER) */
    int32_t system;       /* WCNST_ADVECTION / WCNST_BURGERS / WCNST_EULER */
    int32_t nx, ny;       /* unknowns per direction, >= 5 (ny = 1 in 1D) */
    double x0, x1;        /* domain; spacing dx = (x1 - x0) / nx */
    double y0, y1;        /* dy = (y1 - y0) / ny in 2D */
    int32_t bc_x, bc_y;   /* WCNST_PERIODIC / WCNST_ZERO_GRADIENT / WCNST_REFLECT (Euler: mirror
                             image, normal momentum reversed) / WCNST_FIXED (ghosts hold
                             fixed_x / fixed_y) */
    int32_t flux;         /* WCNST_ROE (no entropy fix) / WCNST_LF (local) /
                             WCNST_VANLEER (flux-vector splitting, Euler only) */
    int32_t scheme;       /* WCNST_TENO (Eqs. 16-19) / WCNST_LINEAR (Eq. 12) / WCNST_JS (Eq. 14) /
                             WCNST_Z (the WCNS-Z of Sec. 3: weights of Borges et al. 2008 on the
                             indicators of Eq. 15 and tau_5 of Sec. 2.3) */
    int32_t diff;         /* WCNST_MND (Eq. 5) / WCNST_MD (Eq. 3) / WCNST_HWCNS (Eq. 4); MD and
                             HWCNS: 1D single solves only (batches and pools use MND) */
    int32_t charwise;     /* Euler: 1 = interpolate characteristic variables */
    int32_t q;            /* TENO integer power, Eq. (16), in [1, 64]; default 6.  The cut
                             test scales C + tau_5/(beta_k + eps) by a power of two so that the
                             powers cannot overflow, except for q = 6, where they stay finite
                             while C + tau_5/(beta_k + eps) <= 8e50 (tau_5 <= 8e10 with
                             eps = 1e-40) */
    double gamma;         /* ratio of specific heats, > 1; default 1.4 */
    double adv_speed;     /* advection speed a (flux f = a u) */
    double CT;            /* TENO cut-off C_T, Eq. (18); default 1e-5 */
    double C;             /* TENO constant C, Eq. (16); default 1 */
    double eps_teno;      /* TENO epsilon, Eq. (16); default 1e-40 */
    double eps_js;        /* Jiang-Shu epsilon, Eq. (14); default 1e-6 */
    double fixed_x[2][4]; /* WCNST_FIXED ghost states at x0 / x1, conserved variables in storage
                             order (rho, rho u, [rho v], E; scalars use [0]); default 0 */
    double fixed_y[2][4]; /* ... at y0 / y1 (2D) */
    double gravity;       /* 2D Euler body force in +y: R += (0, 0, rho g, rho v g); default 0 */
    int32_t z_q;          /* WCNST_Z: power p in alpha_k = d_k (1 + (tau_5/(beta_k + eps_z))^p),
                             in [1, 4] (finite for tau_5 < 1e37 with eps_z = 1e-40); default 1 */
    double eps_z;         /* WCNST_Z: epsilon, > 0; default 1e-40 */
} wcnst_desc;

typedef struct wcnst_solver wcnst_solver;

/* Fill *d with the paper's defaults: 1D Euler, Roe, TENO, MND, charwise,
 * gamma 1.4, C_T 1e-5, C 1, q 6, eps 1e-40, zero-gradient, domain [0, 1];
 * for WCNS-Z p = 1 and eps_z = 1e-40. */
wcnst_status wcnst_desc_init(wcnst_desc* d);

/* Device workspace bytes needed by a solver for *d (control block, two
 * Runge-Kutta stage buffers and, in 2D, 33 KB of segment-layout tables).
 * Returns WCNST_E_INVALID_ARG for a bad desc. */
wcnst_status wcnst_workspace_size(const wcnst_desc* d, size_t* bytes);

/* Validate *d and create a handle bound to hip_stream (a hipStream_t; NULL is
 * the default stream) and to the caller-owned device workspace (256-byte
 * aligned, at least wcnst_workspace_size bytes).  Time and step counters
 * start at 0.  The handle is owned by the library: free it with
 * wcnst_destroy. */
wcnst_status wcnst_create(const wcnst_desc* d, void* hip_stream, void* workspace,
                          size_t ws_bytes, wcnst_solver** out);

/* Discrete right-hand side R = -(dF/dx + dG/dy) of Eq. (2) for the state U
 * (Sec. 2.1 Eq. (5), or Eq. (3) for WCNST_MD, on midpoint fluxes from
 * Sec. 2.2-2.3), ghost cells filled by the boundary conditions.  U and R
 * are device arrays of nvar*ny*nx doubles and must not overlap.
 * Asynchronous.
 * flags (nullable, device, uint8): the stencil-cut pattern of every
 * interpolation, direction x first then y:
 *   x block [nvar][ny][nx+3][2], y block [nvar][nx][ny+3][2];
 *   with WCNST_MD (1D) the one block is [nvar][1][nx+5][2], with
 *   WCNST_HWCNS [nvar][1][nx+1][2];
 * entry [k][line][s][side] is for the midpoint x_{j+1/2}, j = s - 2 (MND),
 * j = s - 3 (MD) or j = s - 1 (HWCNS), of
 * characteristic field k (conserved variable k when charwise = 0; for y
 * lines the normal momentum comes first), side 0 = u_L, side 1 = u_R
 * (mirrored stencil); bit k-1 holds delta_k of Eq. (18).  Schemes without
 * a cut (LINEAR, JS, Z) report 7. */
wcnst_status wcnst_rhs(wcnst_solver* s, const double* U, double* R, uint8_t* flags);

/* One SSP-RK3 step of U in place (Sec. 2, Shu-Osher form).  dt > 0 is used
 * as given; dt <= 0 takes dt = cfl / max((|u|+c)/dx [+ (|v|+c)/dy]) from U
 * (|a|/dx for advection, |u|/dx for Burgers).  Asynchronous; advances the
 * device time by dt.  A non-physical stage output sets the sticky status. */
wcnst_status wcnst_step(wcnst_solver* s, double* U, double dt, double cfl);

/* Advance U in place from the current device time until t_final (dt clipped
 * so the last step lands on it; stops once t_final - t <= 1e-12 t_final) or
 * for max_steps steps when t_final is +inf.  Synchronous at return.
 * Returns WCNST_E_NONPHYSICAL (see wcnst_status_sync for where) or
 * WCNST_E_MAX_STEPS when t_final was not reached in max_steps steps.
 * t_out / steps_out (nullable) receive the device time and the steps taken
 * by this call. */
wcnst_status wcnst_solve(wcnst_solver* s, double* U, double t_final, double cfl,
                         int64_t max_steps, double* t_out, int64_t* steps_out);

/* Largest scratch (bytes) of wcnst_solve_noalloc: the control block and two
 * stage buffers, 256 + 2 x nvar x nx x ny x 8 bytes rounded to 256 each;
 * 64 MiB admits 2D grids up to 1024 x 1023 (about 1.05e6 cells) and 1D
 * Euler lines up to 1.39e6 cells. */
#define WCNST_NOALLOC_MAX_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of wcnst_solve, from t = 0, on a grid described by *d, with the control
 * block and the stage buffers in a static device array of
 * WCNST_NOALLOC_MAX_BYTES that the library holds on each device it runs on
 * (no handle, no workspace, no pinned host memory; nothing is allocated).
 * U (device, [nvar][ny][nx] FP64, caller-owned) is advanced in place on
 * hip_stream until t_final (or for max_steps steps when t_final is +inf),
 * with the same kernels and results as wcnst_solve.  Synchronous at return.
 * t_out / steps_out (nullable) receive the time reached and the steps taken.
 * Returns WCNST_E_INVALID_ARG for a bad descriptor or a grid whose scratch
 * would exceed the limit (before any device work), WCNST_E_NONPHYSICAL /
 * WCNST_E_MAX_STEPS as wcnst_solve.  Every call on one device shares that
 * device's array, which keeps the last call's contents (each call resets
 * what must start at zero): calls that overlap on one device, from several
 * host threads or streams, race. */
wcnst_status wcnst_solve_noalloc(const wcnst_desc* d, void* hip_stream, double* U, double t_final,
                                 double cfl, int64_t max_steps, double* t_out, int64_t* steps_out);

/* Synchronise the stream and read the device counters: time, total steps,
 * sticky status, and for WCNST_E_NONPHYSICAL the global stage index
 * (3*step + stage) and the cell (y*nx + x) of the first offending value
 * (-1 when none).  Any pointer may be NULL. */
wcnst_status wcnst_status_sync(wcnst_solver* s, double* t, int64_t* steps, int32_t* status,
                               int64_t* bad_stage, int64_t* bad_cell);

/* Reset the device time, step counter and sticky status (asynchronous). */
wcnst_status wcnst_reset(wcnst_solver* s, double t, int64_t steps);

/* Launch shape of the 2D stage kernel: one 64-lane wavefront per strip of
 * 61 columns marches up a segment of rows_per_segment rows (>= 1).  The
 * default, chosen at wcnst_create from the grid and the device's CU count,
 * is in [2, 35]: 35 rows for grids that fill the device, shorter segments
 * (more wavefronts) for smaller ones; 0 restores it.  Changes only the work
 * decomposition, never the results.  Negative values: WCNST_E_INVALID_ARG. */
wcnst_status wcnst_set_tuning(wcnst_solver* s, int32_t rows_per_segment);

/* Launch shape of the stage kernels (wcnst_step / wcnst_solve).  2D: strips
 * of 61 columns; segments 0 .. nseg1-1 of each strip hold rows1 rows, the
 * later ones (to nseg in all, the last one ragged) rows2.  Two heights are
 * used only without an explicit tuning, for a launch of one round with two
 * wavefronts on most SIMDs: a SIMD issues from its oldest wavefront first,
 * and the first-dispatched segments get more rows so that both wavefronts
 * finish together.  1D: strips only (rows and segments 1).  Right-hand-side
 * launches use one height. */
wcnst_status wcnst_stage_shape(const wcnst_solver* s, int32_t* strips, int32_t* rows1, int32_t* rows2,
                               int32_t* nseg1, int32_t* nseg);

/* Rows of the first-height segments in the next two-height 2D stage launch.
 * Those segments do not keep rows1 rows each: every launch records how long
 * each took, and the launch after next moves rows from the segments that
 * took longer (where the stencil-cut test of Sec. 2.3 runs in full, near
 * discontinuities) to the others, so that all wavefronts finish about
 * together; the first nseg1 * rows1 rows of a strip stay theirs.  Only the
 * decomposition changes, never the results.  On return *count is strips *
 * (nseg1 + 1), the boundaries [strip][0 .. nseg1] (row 0 up to nseg1 *
 * rows1), or 0 where stage launches use fixed heights (1D, one height, a
 * tuning set, the allocation-free solve).  rows (host, nullable): filled
 * when cap >= *count, after the solver's stream has drained. */
wcnst_status wcnst_stage_layout(wcnst_solver* s, int32_t* rows, int32_t cap, int32_t* count);

/* Kernel timing for roofline reports: when enabled, every stage kernel is
 * bracketed by HIP events on the solver's stream.  wcnst_profile_read
 * synchronises and returns the summed stage-kernel milliseconds and the
 * number of stage-kernel launches since the last reset. */
wcnst_status wcnst_profile_enable(wcnst_solver* s, int enable);
wcnst_status wcnst_profile_read(wcnst_solver* s, double* stage_ms, int64_t* stage_launches);

/* Free the handle (host state only; the workspace stays the caller's). */
wcnst_status wcnst_destroy(wcnst_solver* s);

/* ---------------------------------------------------------------- batches
 * Many independent 1D Euler problems of uneven length advanced together in
 * ticks: a tick is a chunk of SSP-RK3 steps, each stage one launch covering
 * the strips of every instance still running (own control block, dt and
 * step parity per instance), captured in a HIP graph and replayed while the
 * set of running instances is unchanged; between ticks finished instances
 * drop out of the launch table.  Every instance follows exactly the
 * arithmetic of wcnst_solve (Sec. 2-3 as above), so it gives the same bits
 * batched as alone.  All descriptors must be 1D Euler with the same scheme
 * parameters (flux, scheme, charwise, q, gamma, C_T, C, eps); nx, the domain
 * and the boundary conditions may differ.
 *
 * States live in one packed device buffer of FP64: instance i occupies
 * offsets[i] .. offsets[i] + 3*nx_i - 1 with layout [v][nx_i]
 * (wcnst_batch_offsets; offsets[n] is the buffer length in doubles). */
typedef struct wcnst_batch wcnst_batch;
typedef struct wcnst_pool wcnst_pool;

/* Device workspace bytes for a batch of n descriptors (launch table,
 * control blocks, two packed stage buffers). */
wcnst_status wcnst_batch_workspace_size(const wcnst_desc* descs, int32_t n, size_t* bytes);

/* Validate and create a batch bound to hip_stream and to a caller-owned
 * 256-byte-aligned workspace.  The handle is owned by the library. */
wcnst_status wcnst_batch_create(const wcnst_desc* descs, int32_t n, void* hip_stream, void* workspace,
                                size_t ws_bytes, wcnst_batch** out);

/* Host array of n + 1 element offsets into the packed state buffer. */
wcnst_status wcnst_batch_offsets(const wcnst_batch* b, int64_t* offsets);

/* Advance every instance of the packed device buffer U in place from t = 0
 * to t_final[i] (host array; +inf means exactly max_steps steps) with the
 * CFL rule of wcnst_solve.  Synchronous.  status, t_out, steps_out are host
 * arrays of n (t_out / steps_out nullable); status[i] is WCNST_OK,
 * WCNST_E_NONPHYSICAL or WCNST_E_MAX_STEPS and the return value is the first
 * non-zero one. */
wcnst_status wcnst_batch_solve(wcnst_batch* b, double* U, const double* t_final, double cfl, int64_t max_steps,
                               int32_t* status, double* t_out, int64_t* steps_out);

/* For each instance of the last solve: global stage (3*step + stage) and
 * cell of the first non-physical value, or -1 (host arrays of n). */
wcnst_status wcnst_batch_bad_cells(const wcnst_batch* b, int64_t* bad_stage, int64_t* bad_cell);

/* Steps per tick (even, in [2, 4096], default 64): how often finished
 * instances leave the launch table.  Never changes results. */
wcnst_status wcnst_batch_set_tuning(wcnst_batch* b, int32_t steps_per_tick);

/* Persistent finish (Sec. 2 arithmetic unchanged): once the instances still
 * running hold at most switch_strips strips of 61 cells, the batch stops
 * issuing ticks and runs them to their final times in one persistent launch:
 * each workgroup of waves_per_group wavefronts (1..8) owns
 * instances_per_group instances (1..8), keeps their step control in LDS and
 * shares their strips among its waves stage by stage, ordered by workgroup
 * barriers only (no workgroup waits for another).  switch_strips = 0 (the
 * default) keeps ticks to the end.  Never changes results. */
wcnst_status wcnst_batch_set_persist(wcnst_batch* b, int32_t switch_strips, int32_t waves_per_group,
                                     int32_t instances_per_group);

/* Device time in milliseconds of the last wcnst_batch_solve, from its first
 * launch to the end of its last tick (HIP events on the batch's stream). */
wcnst_status wcnst_batch_kernel_ms(const wcnst_batch* b, double* ms);

/* Ticks of the last wcnst_batch_solve, graphs captured for them, and the
 * instances it finished in a persistent launch (all nullable). */
wcnst_status wcnst_batch_stats(const wcnst_batch* b, int32_t* ticks, int32_t* graphs, int32_t* persist_instances);

wcnst_status wcnst_batch_destroy(wcnst_batch* b);

/* ------------------------------------------------------------ request pools
 * A pool keeps many independent Euler solves (1D and 2D, any sizes, one
 * scheme) resident on the device and advances them together in ticks, so
 * that requests join and leave between ticks (continuous batching).  Each
 * request follows exactly the arithmetic of wcnst_solve (Sec. 2-3, SSP-RK3
 * with the CFL rule and final-step clipping), so its result is the same
 * bits alone or in any mix.  A tick issues, per dimension, one stage
 * launch per Runge-Kutta stage covering all active grids of that dimension
 * (each with its own control block and dt); no wave waits for another.
 * The library allocates no device memory: the
 * pool's tables live in a caller workspace and every request brings its own
 * three state buffers.
 *
 * Bytes of the device workspace of a pool for `capacity` requests. */
wcnst_status wcnst_pool_workspace_size(int32_t capacity, size_t* bytes);

/* Create a pool for Euler requests with the scheme parameters of `scheme`
 * (its sizes are ignored) on hip_stream (1D passes and result copies; the
 * pool adds one stream of its own, default priority, for 2D launches). */
wcnst_status wcnst_pool_create(const wcnst_desc* scheme, int32_t capacity, void* hip_stream, void* workspace,
                               size_t ws_bytes, wcnst_pool** out);

/* Admit a request: U holds its initial state ([nvar][ny][nx] FP64, nvar =
 * 3 in 1D, 4 in 2D) and, with U1 and U2 of the same size, stays owned by
 * the caller and must not be touched until the request is released.  The
 * state at t = 0 must be in U before the next tick starts on hip_stream.
 * t_final must be finite.  Returns the slot, or WCNST_E_INVALID_ARG when
 * the pool is full or d does not match the pool's scheme. */
wcnst_status wcnst_pool_admit(wcnst_pool* p, const wcnst_desc* d, double* U, double* U1, double* U2,
                              double t_final, double cfl, int32_t* slot);

/* One tick: every admitted, unfinished request advances by up to `steps`
 * steps (fewer when it reaches t_final or a non-physical state).
 * Synchronous.  n_active (nullable) = requests that were advanced. */
wcnst_status wcnst_pool_tick(wcnst_pool* p, int64_t steps, int32_t* n_active);

/* As wcnst_pool_tick with separate step counts for the 1D and the 2D
 * requests (their launches run side by side on two streams, so a caller
 * can give each about the same device time per tick).  Each request's
 * result does not depend on the step counts. */
wcnst_status wcnst_pool_tick_split(wcnst_pool* p, int64_t steps_1d, int64_t steps_2d, int32_t* n_active);

/* Device time (ms, HIP events) from the start of the last tick to the end
 * of its 1D launches and to the end of its 2D launches; 0 for a dimension
 * with no active request. */
wcnst_status wcnst_pool_tick_ms(const wcnst_pool* p, double* ms_1d, double* ms_2d);

/* Outcome of the request in `slot` after the last tick: finished (t_final
 * reached or failed), status (WCNST_OK or WCNST_E_NONPHYSICAL), t, steps,
 * and the global stage and cell of the first non-physical value (-1 when
 * none).  All outputs nullable. */
wcnst_status wcnst_pool_result(const wcnst_pool* p, int32_t slot, int32_t* finished, int32_t* status, double* t,
                               int64_t* steps, int64_t* bad_stage, int64_t* bad_cell);

/* Free the slot (the request's buffers return to the caller). */
wcnst_status wcnst_pool_release(wcnst_pool* p, int32_t slot);

/* Rows per 2D segment of the pool's stage launches (>= 1), or 0 for the
 * default: chosen per tick, as at wcnst_create, over all active 2D
 * requests.  Never changes results. */
wcnst_status wcnst_pool_set_tuning(wcnst_pool* p, int32_t rows_per_segment);

wcnst_status wcnst_pool_destroy(wcnst_pool* p);

/* Message of the last error on this thread ("" when none). */
const char* wcnst_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
