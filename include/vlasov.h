/*
 * vlasov.h - C ABI of the MI355X (gfx950) solver for the one-dimensional
 * Vlasov equation with long-range mean-field forces, after T. M. Rocha Filho,
 * "Solving the Vlasov equation for one-dimensional models with long range
 * interactions on a GPU" (arXiv:1206.3229).
 *
 * The distribution f(x, p, t) lives on an nx-by-np grid in device memory,
 * row-major f[j*nx + i] with i the position index and j the momentum index
 * (the layout of Sec. 3).  Axis u in [umin, umax) has nodes
 * u_k = umin + k*du, du = (umax - umin)/n.  One time step is the time split of
 * Sec. 3, steps 1-4 (eqs. step1-step4): half drift in x, mean-field force from
 * the drifted f (eq. step2), full kick in p, half drift in x.  Every sweep
 * evaluates the cubic spline of eqs. (splinegen, splinecoeffs) at the foot of
 * the characteristic with second derivatives from the eighth-order stencil of
 * eq. (findif).  Options of vlasov_params: the global spline of eq.
 * (tridiagsys) in place of the stencil (the paper's comparison baseline), and
 * the fourth-order compositions of the step and the filter in p that the
 * conclusions name as extensions.
 *
 * Conventions for every call:
 *   - Status: 0 (VLASOV_OK) on success, VLASOV_PENDING (1) from poll only,
 *     a negative VLASOV_E_* code on failure.  vlasov_last_error() returns the
 *     message of the last failure on the calling thread.
 *   - Device memory is owned by the caller (the library never allocates device
 *     memory): the f pair, the workspace and the server arena are passed in as
 *     plain device pointers, 256-byte aligned, and must outlive the context.
 *   - hip_stream is a hipStream_t passed as void* (NULL: the null stream).
 *     Work is enqueued asynchronously on it; only calls that return host data
 *     synchronise it.
 *   - Host buffers are read during the call only, and written only on success.
 *   - A context is not thread-safe; a server is (submit and poll may be called
 *     from any thread).
 *   - A failed call leaves the context as it was, except after VLASOV_E_HIP.
 */
#ifndef VLASOV_H
#define VLASOV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VLASOV_OK = 0,
    VLASOV_PENDING = 1,
    VLASOV_E_INVAL = -1,     /* invalid argument */
    VLASOV_E_NOMEM = -2,     /* request larger than the whole server arena */
    VLASOV_E_HIP = -3,       /* a HIP runtime error (message has its string) */
    VLASOV_E_STATE = -4,     /* call not valid in the current state */
    VLASOV_E_NOTFOUND = -5,  /* unknown ticket */
    VLASOV_E_NONFINITE = -6  /* a diagnostic came out NaN or infinite */
};

/* Pair potentials of Sec. 2: HMF (eq. hmfpot), ring (eq. ringpot) and
 * self-gravitating sheets (eq. sheetpot, with V = 2 pi G |x|), plus a fixed
 * force F(x) given by the caller. */
typedef enum {
    VLASOV_MODEL_HMF = 0,
    VLASOV_MODEL_RING = 1,
    VLASOV_MODEL_SHEET = 2,
    VLASOV_MODEL_EXTERNAL = 3
} vlasov_model;

/* Storage of f between sweeps.  Densities, forces, foot positions and all
 * diagnostics are computed in FP64 for both. */
typedef enum { VLASOV_F64 = 0, VLASOV_F32 = 1 } vlasov_storage;

/* Boundary of an axis: periodic, or zero extension (every sample outside the
 * grid reads 0; mass advected out of the box is lost). */
typedef enum { VLASOV_BC_PERIODIC = 0, VLASOV_BC_ZERO = 1 } vlasov_bc;

/* How f'' of the cubic spline of eq. (splinegen) is obtained. */
typedef enum { VLASOV_SPLINE_FD = 0, VLASOV_SPLINE_GS = 1 } vlasov_spline;

/* Time splitting (the higher-order schemes the conclusions name as an
 * extension).  A step of size dt applies the Sec. 3 step (half drift, force,
 * kick, half drift) with the sizes w_k dt in turn:
 *   STRANG      w = (1), the paper's scheme, second order;
 *   TRIPLE_JUMP w = (w1, w0, w1), w1 = 1/(2 - 2^(1/3)), w0 = 1 - 2 w1
 *               (Yoshida; Forest and Ruth), fourth order;
 *   SUZUKI      w = (p, p, 1 - 4p, p, p), p = 1/(4 - 4^(1/3)), fourth order
 *               with a smaller error constant.
 * Each w_k is the double nearest to the exact value.  The drifts of
 * consecutive substeps are separate sweeps (run fused in one kernel where
 * possible, like those of consecutive steps). */
typedef enum { VLASOV_SPLIT_STRANG = 0, VLASOV_SPLIT_TRIPLE_JUMP = 1, VLASOV_SPLIT_SUZUKI = 2 } vlasov_splitting;

typedef struct {
    int32_t model;    /* vlasov_model */
    int32_t storage;  /* vlasov_storage */
    int32_t bc_x;     /* vlasov_bc; HMF and ring require periodic */
    int32_t bc_p;     /* vlasov_bc */
    int64_t nx, np;   /* grid points, 16 <= n <= 2^19 each, nx*np < 2^31 */
    double xmin, xmax, pmin, pmax;
    double dt;        /* time step, finite and nonzero */
    double ring_eps;  /* softening of eq. (ringpot), > 0 (ring only) */
    double sheet_G;   /* coupling of the sheet model, F = 2 pi G (M(>x) - M(<x)) */
    int64_t hist_cap; /* entries kept of the magnetization history, one per force
                         evaluation (>= 0) */
    int32_t spline;   /* VLASOV_SPLINE_FD: f'' by the local stencil of eq. (findif);
                         VLASOV_SPLINE_GS: the global spline of eq. (tridiagsys), the
                         paper's baseline (lines of at most 4096 samples, single contexts
                         only: batches and the server reject it) */
    int32_t splitting;    /* vlasov_splitting */
    int32_t filter_every; /* 0: no filter; k > 0: after the last kick of every k-th step
                             (counted from vlasov_init), f <- f - (sigma/256) d^8 f along
                             each column, d^8 the eighth central difference in p (mode
                             kappa damped by 1 - sigma sin^8(kappa/2); mass and every
                             p-moment below degree 8 kept) */
    int32_t reserved;     /* 0 */
    double filter_strength; /* sigma, in (0, 1] when filter_every > 0 */
} vlasov_params;

/* Diagnostics of the current f (rectangle rule on the grid):
 * mass = int f, momentum = int p f, kinetic = int p^2/2 f, potential W of the
 * model (HMF (M^2_0 - M_x^2 - M_y^2)/2 with M_0 the mass; ring and sheet the
 * double sum 1/2 int int V(x-x') rho rho'; external 0), energy = kinetic + W,
 * (mx, my) the magnetization of eq. (mxmydef) (HMF and ring; 0 otherwise),
 * l2 = int f^2 and entropy = -int f log f over the points where f > 0 (Casimirs
 * of eq. casimirs), neg_mass = int f over the points where f < 0 (the spline
 * overshoot).  Every quantity but the entropy is computed in a fixed order of
 * summation (64 interleaved partial sums per line, then a pairwise tree; column
 * sums over 16-row blocks first), independent of the launch shape, so results
 * repeat bit for bit; the entropy uses the device's log. */
typedef struct {
    double mass, momentum, kinetic, potential, energy, mx, my, l2, entropy, neg_mass;
} vlasov_moments_t;

typedef struct vlasov_ctx vlasov_ctx;

/* ---------------------------------------------------------------------------
 * Single simulation.
 * ------------------------------------------------------------------------- */

/* Bytes of the device f pair: 2 * nx * np * (8 for F64, 4 for F32).  0 if the
 * parameters are invalid. */
size_t vlasov_f_bytes(const vlasov_params *p);

/* Bytes of the device workspace (line tables, density partial sums, density,
 * force, magnetization history, diagnostics).  0 if invalid. */
size_t vlasov_workspace_bytes(const vlasov_params *p);

/* Create a context.  f0_host: nx*np FP64 values, row-major [np][nx], copied
 * (rounded to nearest FP32 for F32 storage); NULL leaves f unset (then
 * vlasov_generate_ic or vlasov_write_f gives it).  f_dev: vlasov_f_bytes() bytes;
 * ws_dev: vlasov_workspace_bytes() bytes.  Builds the drift line tables
 * (constant over the run) and the model tables on the host and uploads them.
 * Synchronises hip_stream before returning.  Errors: VLASOV_E_INVAL for bad
 * parameters (see vlasov_params), NULL or misaligned pointers; VLASOV_E_HIP. */
int vlasov_init(const vlasov_params *p, const double *f0_host, void *f_dev, void *ws_dev, void *hip_stream,
                vlasov_ctx **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * vlasov_init, but the workspace is the library's static device array of
 * 16 MiB (one per device, held from its first use until the process ends)
 * instead of a caller buffer; the caller still passes f0_host and the f pair
 * f_dev (memory of the current device).  The call allocates nothing: no
 * hipMalloc, hipFree or other allocating routine.  It rejects parameters
 * whose vlasov_workspace_bytes() exceed 16 MiB with VLASOV_E_INVAL (every grid
 * up to 4096 x 4096 fits; 8192 x 4096 does not).  One context per device may
 * hold the array at a time: a second vlasov_init_static on the same device
 * before vlasov_destroy of the first returns VLASOV_E_STATE (two contexts on
 * one array would race).  Everything the step reads is rewritten at init, so
 * the contents left by an earlier context do not matter.  Errors otherwise as
 * vlasov_init; VLASOV_E_INVAL also if f_dev is not memory of the current
 * device. */
int vlasov_init_static(const vlasov_params *p, const double *f0_host, void *f_dev, void *hip_stream,
                       vlasov_ctx **out);

/* EXTERNAL model only: set the force F(x_i), nx FP64 values (copied).
 * VLASOV_E_STATE on other models. */
int vlasov_set_external_force(vlasov_ctx *c, const double *F_host);

/* Enqueue nsteps (>= 0) time steps of Sec. 3 (steps 1-4), each made of the
 * substeps of params.splitting, and the filter of params.filter_every.
 * Consecutive half drifts of successive (sub)steps are fused into one pass
 * over f; the result is bit-identical to nsteps separate steps. */
int vlasov_step(vlasov_ctx *c, int64_t nsteps);

/* Steps that are not the last of a vlasov_step call are enqueued
 * steps_per_graph at a time as one HIP graph launch (default 0: every kernel
 * launched on its own, which measured faster on the 4096^2 sheet).  The graph of a context is captured the first
 * time it is needed (once for each of the two buffers f may start in) and
 * replayed afterwards; its kernels are those of the eager path, so results are
 * identical bit for bit.  Graphs are not used while the per-kernel timers are
 * on or with the filter.  Synchronises the stream when the value changes;
 * VLASOV_E_INVAL outside [0, 4096]. */
int vlasov_set_graph(vlasov_ctx *c, int32_t steps_per_graph);

/* The individual sweeps of a step, for inspection and testing (with the
 * sizes of the first substep: dt itself for the Strang splitting).
 * vlasov_drift: npass (1 or 2) successive half drifts (eqs. step1/step4) of
 *   the current f, tau = w_0 dt/2 each; also leaves the density partial sums
 *   of the result.
 * vlasov_force: density of the current f and the model force (eq. step2);
 *   writes F (nx values) and the magnetization (2 values) to the host if the
 *   pointers are non-NULL (then synchronises), and keeps F for the kick.
 * vlasov_kick: the momentum advection of eq. (step3) with the last force;
 *   VLASOV_E_STATE if no force was computed yet. */
int vlasov_drift(vlasov_ctx *c, int32_t npass);
int vlasov_force(vlasov_ctx *c, double *F_host, double *mxmy_host);
int vlasov_kick(vlasov_ctx *c);

/* Diagnostics of the current f; synchronises.  VLASOV_E_NONFINITE (out still
 * written) if any value is NaN or infinite. */
int vlasov_moments(vlasov_ctx *c, vlasov_moments_t *out);

/* Magnetization (M_x, M_y) of the drifted f used by each force evaluation
 * (HMF and ring; one per substep), oldest first.  Copies min(count, cap,
 * hist_cap) entries, sets *count to the number of evaluations recorded so
 * far; synchronises. */
int vlasov_mag_history(vlasov_ctx *c, double *mx, double *my, int64_t cap, int64_t *count);

/* Copy the current f to the host as FP64 [np][nx]; synchronises. */
int vlasov_read_f(vlasov_ctx *c, double *f_host);

/* Replace the current f (checkpoint restore), FP64 [np][nx]; synchronises.
 * The step count of the filter schedule is not changed. */
int vlasov_write_f(vlasov_ctx *c, const double *f_host);

/* Initial conditions the library generates on the device (the paper's
 * workloads, Sec. 4), every one normalised to unit mass on the grid: the raw
 * values r_ij are summed in index order (each row from i = 0, then the row
 * sums from j = 0) to S, and f_ij = r_ij / ((S dx) dp) (rounded to FP32 for F32
 * storage).  Nodes u_k = umin + k du.
 *   WATERBAG     r = 1 on |x_i| <= a0, |p_j| <= a1 (inclusive; each half-width
 *                raised to at least two cells), else 0; with amp != 0 the
 *                support values are 1 + amp eta_k, eta_k = 2 u_k - 1, u_k the
 *                top 53 bits of output k = j nx + i of the SplitMix64 stream of
 *                `seed` (Steele, Lea and Flood 2014: z = seed + (k + 1)
 *                0x9E3779B97F4A7C15, then the mix with shifts 30, 27, 31 and
 *                multipliers 0xBF58476D1CE4E5B9, 0x94D049BB133111EB) times 2^-53.
 *   WATERBAG_UM  the HMF waterbag of magnetization M0 = a1 in [0, 1) and energy
 *                per particle U = a0 (Sec. 4.2): theta0 solves sin(t)/t = M0
 *                (bisection on (0, pi), at most 200 halvings, until hi - lo <=
 *                4e-16 hi; theta0 the midpoint), p0 = sqrt(6 (U - (1 - M0^2)/2));
 *                then WATERBAG with half-widths (theta0, p0).
 *   GAUSSIAN     r = exp(-p_j^2 / (2 a0)) (1 + amp cos(x_i - phi)) with a0 = T > 0,
 *                |amp| < 1, phi = 0 for seed 0, else 2 pi u_0; exp and cos are
 *                the host C library's, evaluated once per node. */
typedef enum {
    VLASOV_IC_HOST = 0,  /* f0 comes from the caller (requests only) */
    VLASOV_IC_WATERBAG = 1,
    VLASOV_IC_WATERBAG_UM = 2,
    VLASOV_IC_GAUSSIAN = 3
} vlasov_ic_kind;

typedef struct {
    int32_t kind;  /* vlasov_ic_kind */
    int32_t reserved;
    double a0, a1, amp;
    uint64_t seed;
} vlasov_ic;

/* Replace the current f by a generated initial condition (device kernels on
 * the context's stream); synchronises.  VLASOV_E_INVAL for an unknown kind or
 * parameters outside the ranges above (checked before anything runs), or if
 * the raw values sum to zero (no node in the support; f is then undefined). */
int vlasov_generate_ic(vlasov_ctx *c, const vlasov_ic *ic);

/* Release the context (host memory only; caller device memory is untouched).
 * Synchronises the stream first. */
int vlasov_destroy(vlasov_ctx *c);

/* Message of the last failing call on this thread ("" if none). */
const char *vlasov_last_error(void);

/* ---------------------------------------------------------------------------
 * Launch shapes.  Every shape computes the same arithmetic (results are
 * bit-identical); they differ only in speed, which the autotuner measures.
 * ------------------------------------------------------------------------- */

typedef struct {
    int32_t drift_threads;     /* threads per drift workgroup: 64, 128 or 256 (2 columns each) */
    int32_t kick_rows;         /* rows per thread of the kick: 8, 16 or 32 */
    int32_t kick_drift_width;  /* 0: the kick (step 3) and the two half drifts after it (step 4
                                  and the next step 1) run as separate kernels; 230 or 486: one
                                  fused kernel on tiles of that many columns (four or eight
                                  wavefronts: the 256 or 512 columns a tile kicks, one per
                                  thread), which reads and writes f once for the three sweeps.
                                  It is used where the combined drift offsets of the rows of
                                  every tile differ by at most 8 columns, else the separate
                                  kernels run.  The last step of a call (kick and one half
                                  drift) always uses the separate kernels. */
    int32_t kick_drift_blocks; /* rows of a fused tile in 16-row density blocks: 1 to 4 */
} vlasov_tuning;

/* The compiled launch shapes: writes min(cap, total) of them, *n = total. */
int vlasov_tuning_candidates(vlasov_tuning *out, int32_t cap, int32_t *n);

/* Select a compiled launch shape for a context (VLASOV_E_INVAL otherwise).
 * Defaults: 128 drift threads, 16 (FP64) or 32 (FP32) kick rows, fused kick
 * and drift on tiles of 230 columns by 32 rows where the grid gives at least
 * 2048 such tiles, else by 16 rows.  Changing kick_drift_blocks
 * rebuilds the fused tables (synchronises the context's stream). */
int vlasov_set_tuning(vlasov_ctx *c, const vlasov_tuning *t);
int vlasov_get_tuning(vlasov_ctx *c, vlasov_tuning *t);

/* ---------------------------------------------------------------------------
 * Batches: many contexts stepped together (one persistent launch per phase).
 * ------------------------------------------------------------------------- */

#define VLASOV_BATCH_MAX 256

/* Flags of batched stepping and of the server (the `flags` arguments):
 *   VLASOV_BATCH_GRAPH  capture the chunk's launches into a HIP graph once and
 *                       replay it;
 *   VLASOV_BATCH_FUSE   run each member's kick fused with the pair of half drifts
 *                       after it (the single-grid fused kernel on 230-column
 *                       tiles, or on 182-column tiles with 56 columns of
 *                       slack for members whose drift offsets spread by 9 to
 *                       56 columns inside a 16-row tile; members with a
 *                       periodic p axis): f is read and written once
 *                       for the three sweeps.  It sets each member's
 *                       kick_drift_blocks to 1 (the batched tiles are 16
 *                       rows tall; synchronises a member whose tuning had
 *                       another value).  Requested by the caller (the
 *                       benchmark's server uses it: faster than the separate
 *                       phases on its 512-request burst). */
enum { VLASOV_BATCH_GRAPH = 1, VLASOV_BATCH_FUSE = 2 };

/* Bytes of device scratch for batched stepping in chunks of chunk_cycles
 * cycles (grid descriptors and per-cycle work tables, two sets). */
size_t vlasov_batch_scratch_bytes(int32_t chunk_cycles);

/* Advance ctxs[k] by nsteps[k] >= 0 time steps (Sec. 3, steps 1-4), for
 * k < n <= VLASOV_BATCH_MAX distinct contexts of one storage type created on one
 * stream; grids may differ in size, model and dt.  Every phase (drift,
 * density, force, kick) of all grids is one persistent launch whose
 * workgroups stride over the tiles of all grids; chunk_cycles cycles are
 * planned at a time and enqueued (flags: VLASOV_BATCH_*).  Each grid's result
 * is bit-identical to vlasov_step on it alone.
 * Batches run the local spline with the Strang splitting and no filter.
 * scratch_dev: vlasov_batch_scratch_bytes(chunk_cycles) bytes, 256-aligned.
 * Synchronises the stream before returning.  VLASOV_E_INVAL for mismatched
 * contexts or a short scratch buffer. */
int vlasov_batch_step(vlasov_ctx *const *ctxs, int32_t n, const int64_t *nsteps, void *scratch_dev,
                      size_t scratch_bytes, int32_t chunk_cycles, int32_t flags);

/* ---------------------------------------------------------------------------
 * Serving: a request loop over parameter-scan simulations of uneven sizes with
 * continuous batching.  Requests wait in FIFO order until a batch slot is free
 * and their footprint fits in the caller's device arena; admitted requests join
 * the running batch at the next chunk boundary, finished ones leave it and free
 * their arena space.  Results equal those of vlasov_step on the request alone.
 * ------------------------------------------------------------------------- */

typedef struct vlasov_server vlasov_server;

typedef struct {
    vlasov_params p;  /* storage must equal the server's; hist_cap must be 0; the
                         local spline with the Strang splitting and no filter */
    int64_t nsteps;   /* >= 0 */
    int32_t keep_f;   /* nonzero: keep the final f for vlasov_poll */
    int32_t reserved;
    vlasov_ic ic;     /* kind VLASOV_IC_HOST: f0 passed to vlasov_submit; any other
                         kind: generated by the server on the device when the
                         request is admitted (part of its latency) */
} vlasov_request;

typedef struct {
    int32_t status;   /* VLASOV_OK, or the failure code of this request */
    int32_t reserved;
    int64_t steps_done;
    double t_submit, t_admit, t_done; /* seconds since the server was created */
    vlasov_moments_t m;               /* diagnostics of the final f */
} vlasov_result;

/* Arena bytes an admitted request occupies (f pair and workspace). 0 if invalid. */
size_t vlasov_request_footprint(const vlasov_params *p);

/* Arena bytes the server reserves for its tables (at the start of the arena). */
size_t vlasov_server_table_bytes(int32_t chunk_cycles);

/* Create a server over the caller's device arena (256-aligned, kept until
 * destroy).  storage: VLASOV_F32 or VLASOV_F64 for every request; max_slots
 * <= VLASOV_BATCH_MAX grids run at once; chunk_cycles cycles per chunk; flags
 * VLASOV_BATCH_*.  A scheduler thread owns all GPU work: chunks on hip_stream,
 * admissions (tables and generated initial conditions) and retirements
 * (diagnostics, final f) on two streams of its own, while the next chunk runs.
 * No HIP call is made before the first request is admitted. */
int vlasov_server_create(void *arena_dev, size_t arena_bytes, void *hip_stream, int32_t storage, int32_t max_slots,
                         int32_t chunk_cycles, int32_t flags, vlasov_server **out);

/* Queue a request (thread-safe, non-blocking).  f0_host: [np][nx] FP64,
 * copied, for r->ic.kind == VLASOV_IC_HOST; ignored (may be NULL) otherwise.
 * VLASOV_E_INVAL for invalid parameters or initial-condition spec,
 * VLASOV_E_NOMEM if the footprint exceeds the whole arena, VLASOV_E_STATE after
 * destroy began. */
int vlasov_submit(vlasov_server *s, const vlasov_request *r, const double *f0_host, uint64_t *ticket);

/* VLASOV_PENDING while queued or running; VLASOV_OK once done: writes the
 * result (and, if the request kept it and f_host is non-NULL, the final f as
 * FP64 [np][nx]) and forgets the ticket.  VLASOV_E_NOTFOUND for an unknown
 * ticket.  Thread-safe. */
int vlasov_poll(vlasov_server *s, uint64_t ticket, vlasov_result *out, double *f_host);

/* Counts of queued, running and finished-but-unpolled requests. */
int vlasov_server_stats(vlasov_server *s, int64_t *queued, int64_t *running, int64_t *done);

/* Drain every queued and running request, stop the scheduler, release host
 * resources.  Unpolled results are discarded. */
int vlasov_server_destroy(vlasov_server *s);

/* ---------------------------------------------------------------------------
 * Measurement.
 * ------------------------------------------------------------------------- */

/* Kernel identifiers for the per-kernel timers. */
enum {
    VLASOV_K_DRIFT = 0,    /* one half drift + density partial sums */
    VLASOV_K_DRIFT2 = 1,   /* two fused half drifts + density partial sums */
    VLASOV_K_DENSITY = 2,  /* density from the partial sums */
    VLASOV_K_FORCE = 3,    /* model force (and magnetization) */
    VLASOV_K_KICK = 4,     /* momentum advection */
    VLASOV_K_MOMENTS = 5,  /* diagnostics */
    VLASOV_K_KICK_DRIFT2 = 6,  /* kick fused with two half drifts + density partial sums */
    VLASOV_K_FILTER = 7,   /* the filter along p (fused with the kick of a filtered step) */
    VLASOV_K_COUNT = 8
};

/* When on, every kernel launch of the context is bracketed by HIP events on
 * its stream.  vlasov_profile_read synchronises, folds the recorded launches
 * of kernel `kernel` into the running totals and returns them (total
 * milliseconds and number of launches since profiling was switched on). */
int vlasov_profile_enable(vlasov_ctx *c, int32_t on);
int vlasov_profile_read(vlasov_ctx *c, int32_t kernel, double *total_ms, int64_t *launches);
const char *vlasov_kernel_name(int32_t kernel);

/* Plain device-to-device copy of `bytes` (multiple of 16) with the library's
 * own streaming kernel, for a measured bandwidth ceiling.  Asynchronous. */
int vlasov_device_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* VLASOV_H */
