/*
 * modap.h -- C ABI of the MI355X (gfx950) pseudo-projection sweep library.
 *
 * The library finds an eps-feasible point of a (possibly changing) system of
 * linear inequalities  A x <= b  with the modified pseudo-projection method
 * (ModAP) of Sokolinsky & Sokolinskaya, "Scalable Parallel Algorithm for
 * Solving Non-stationary Systems of Linear Inequalities":
 *
 *   one sweep at x:   r_i = <a_i, x> - b_i                        (section 2)
 *                     rho+_i = max(r_i, 0)/||a_i||^2 * a_i          (eq. 7)
 *                     y = sum_i rho+_i,  h = #{i : r_i > 0}         (section 3, Map/Reduce)
 *                     dmax = max_i max(r_i, 0)/||a_i||             (eq. 10)
 *   stop when         dmax <= eps_abs                               (eq. 10; see modap_params)
 *   step              x <- x - lambda * y/||y||                     (eq. 12, ModAP)
 *                  or x <- x - (lambda/h) * y                       (Algorithm 1, relaxed;
 *                                                                    phi = y/h, eq. 8)
 *   data update       translation of the feasible set by +v:  b <- b + A v,
 *                     or replacement of rows (a_i, b_i)             (sections 1, 3, 5)
 *
 * Conventions for every entry point:
 *  - Plain C types only; no exception crosses the boundary; every call returns
 *    a modap_status (MODAP_OK = 0).  modap_last_error() gives a message.
 *  - Ownership: caller buffers are only read (or written, for outputs) during
 *    the call -- or, for stream-ordered inputs on the device, by work queued on
 *    the context's stream before the call returns -- and are never retained.
 *    Every device buffer the library uses belongs to the context.
 *  - ptrs_on_device: 0 = caller pointers are host memory; 1 = device memory
 *    of the context's GPU (e.g. torch.Tensor.data_ptr() of a tensor on it).
 *  - Ordering: work is queued on the context's stream in call order.
 *    set_system, set_x, set_drift, update_coeffs and iterate (without stats)
 *    are asynchronous with respect to the host once host inputs are copied;
 *    solve, eval_sweep, query and any call given a stats pointer synchronise.
 *  - Layout: A is dense row-major, row i at A + i*lda elements, lda >= n, in
 *    the storage type; b is m doubles; x, v are n doubles.  BF16 elements are
 *    the upper 16 bits of an IEEE binary32 (uint16 bit patterns).
 *  - Precision: rows are stored as given; ||a_i||^2, b, x, y, the stop test
 *    and the step are FP64.  Dot products accumulate in FP64 for MODAP_F64
 *    storage and in FP32 for MODAP_F32 / MODAP_BF16 storage; the optional
 *    certificate of a stop (modap_params.certify) accumulates in FP64.
 *  - Exact data: the library keeps the right-hand side as bref + A w, with w
 *    the FP64 sum of every translation applied; the sweep carries a working
 *    copy of b translated in its own precision, which the certificate rebases
 *    onto the exact value.
 *  - Threading: a context is used by one host thread at a time; several
 *    contexts may share a device.
 *  - One HIP runtime per process: the library needs libamdhip64.so.7.  In a
 *    process that also uses PyTorch, load PyTorch first (its wheel loads a
 *    HIP runtime of its own by path; loaded after this library it would map
 *    a second one, with which nothing is shared, and calls fail with
 *    E_DEVICE).  The Python binding does this itself.
 *  - Tracing: every working call records a named range on the ROCm tracing
 *    timeline (rocprofv3 --marker-trace), a served request one from its
 *    submission to its end.
 *
 * Environment variables the library reads (all optional):
 *   MODAP_TUNE_CACHE=path        file of autotuned sweep shapes (modap_autotune)
 *   MODAP_RESIDENT=0             small systems iterate in two kernels per
 *                                iteration instead of the resident form
 *   MODAP_RESIDENT_ROWS=k        rows per workgroup the resident form aims for
 *                                (default 32, at least 4)
 *   MODAP_RESIDENT_TIMEOUT_TICKS=t  longest wait of a resident launch at its grid
 *                                barrier, in ticks of the 100 MHz constant clock
 *                                (default 1e8: one second); a longer wait ends the
 *                                launch, and the call reports E_DEVICE
 *   MODAP_BATCH_SHORT=0          batches sweep short rows one to a wavefront
 *                                instead of four
 */
#ifndef MODAP_H
#define MODAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct modap_ctx modap_ctx;

typedef enum {
    MODAP_OK = 0,
    MODAP_E_INVAL = 1,          /* bad argument: sizes, NULL, lda < n, non-finite input, lambda<=0, eps<=0 */
    MODAP_E_ZERO_ROW = 2,       /* a row a_i is zero (section 2 assumes a_i != 0) or not finite */
    MODAP_E_NOMEM = 3,          /* device or pinned-host allocation failed */
    MODAP_E_DEVICE = 4,         /* HIP runtime error; the context must be destroyed */
    MODAP_E_STATE = 5,          /* call before modap_set_system, or the context is broken */
    MODAP_E_NOT_CONVERGED = 6,  /* solve: max_iters steps taken without reaching eps-feasibility */
    MODAP_E_INFEASIBLE = 7,     /* a row is violated but y = 0: no step direction (cannot
                                   happen for a feasible system: <x - z, y> > 0 for z in M) */
    MODAP_E_NUMERIC = 8         /* a NaN or infinity appeared in the iteration */
} modap_status;

typedef enum { MODAP_F64 = 0, MODAP_F32 = 1, MODAP_BF16 = 2 } modap_dtype;

typedef enum {
    MODAP_STEP_FIXED = 0,   /* ModAP, eq. 12: x <- x - lambda*y/||y||  (step of length lambda)  */
    MODAP_STEP_AVG = 1      /* Algorithm 1 relaxed: x <- x - (lambda/h)*y; lambda = 1 is Alg. 1 */
} modap_step;

typedef struct {
    double lambda;          /* > 0: step length (FIXED) or relaxation (AVG) */
    double eps;             /* > 0: stop tolerance */
    int32_t eps_relative;   /* != 0: eps_abs = eps * max_i |b_i| of the current data; else eps_abs = eps */
    int32_t step;           /* modap_step */
    int64_t max_iters;      /* solve: at most this many steps in the call (>= 0) */
    int32_t profile;        /* k > 0: time every k-th iteration's kernels with HIP events recorded
                               by their dispatches (stats); 0: no timing */
    int32_t track;          /* iterate only: != 0 keeps following a changing system -- an
                               eps-feasible check takes no step but does not stop the queued
                               iterations, so drift keeps being applied and re-checked */
    int32_t certify;        /* != 0: every stop at eps-feasibility is confirmed by an FP64
                               certificate before it is accepted (eq. 10 on the exact data):
                               one more pass over the same stored rows with x and the
                               translations in FP64, FP64 accumulation, and a rigorous bound of
                               its own rounding added to every distance.  If the bound exceeds
                               eps_abs, the certificate's y decides a step instead and the
                               iteration goes on.  The certificate also rebases the working
                               right-hand side onto the exact data (see modap_query).  It runs
                               in modap_solve and at the end of modap_iterate, of
                               modap_batch_solve and of a synchronising modap_batch_iterate, and
                               in each round of the server. */
    int32_t pad;
} modap_params;

typedef struct {
    int64_t iters;          /* steps taken since modap_set_system / modap_set_x */
    int64_t sweeps;         /* sweeps (feasibility checks) since then */
    int32_t converged;      /* 1 if the last check found x eps-feasible */
    int32_t state;          /* 0 running, 1 converged, 2 no direction, 3 numeric, 4 step limit, 5 bad row,
                               6 not certifiable (eps_abs below the FP64 certificate's rounding bound) */
    double max_viol;        /* last check: max_i max(r_i, 0)/||a_i|| */
    int64_t h;              /* last check: number of violated rows */
    double y_norm;          /* last check: ||y|| */
    double b_inf;           /* last check: max_i |b_i| */
    double eps_abs;         /* last check: the threshold applied */
    double seconds;         /* host wall time of this call */
    double hbm_bytes;       /* algorithmic bytes of the sweeps launched in this call:
                               m*n*sizeof(A) + 16m (+ 8m when a translation is applied) each */
    double sweep_ms;        /* profile: summed duration of the sweep kernels of this call */
    double reduce_ms;       /* profile: summed duration of the reductions of y (each also makes
                               the previous step permanent in x); the stop decision and the
                               step length are taken at the start of the next sweep */
    int64_t profiled;       /* profile: number of sweeps timed in this call */
    int32_t certified;      /* 1 if the last stop was confirmed by the FP64 certificate (max_viol
                               is then its upper bound of the largest distance) */
    int32_t resident;       /* iterate and solve: 1 if the iterations ran in the resident form (one
                               launch of many iterations, the rows held in LDS, a grid barrier per
                               iteration), 0 if in the two-kernel form; 0 from every other call */
    double b_drift;         /* last certificate: largest |b_i - exact b_i| of the working
                               right-hand side, which the certificate then corrected */
} modap_stats;

/* Kernel shape of the sweep (see modap_set_tile).  kind 0 = one pass with a
 * whole row on chip, kind 1 = split-row two-phase form for very long rows. */
typedef struct {
    int32_t kind;
    int32_t block;          /* threads per workgroup */
    int32_t lanes_per_row;  /* threads that share one row (64 .. block) */
    int32_t chunks;         /* 16-byte vectors per thread per row (kind 0) or per column tile (kind 1) */
    int32_t grid;           /* workgroups of the sweep (0 on input: the library's choice, one per CU) */
    int32_t rows_per_step;  /* rows each row group loads per step */
    int32_t depth;          /* kind 0: steps held per row group; the next depth-1 steps' rows are
                               in flight while one is reduced (0 on input: the library's choice) */
    int32_t interleave;     /* kind 0: 0 = each workgroup takes a contiguous band of rows;
                               1 = the workgroups take consecutive row blocks in turn */
} modap_tile;

/* Create a context on HIP device `device`.  hip_stream: the hipStream_t to
 * queue all work on (the caller keeps it alive for the context's life), or
 * NULL for the device's default (null) stream, which is ordered with the
 * default stream of PyTorch.  Errors: E_INVAL (out == NULL or no such
 * device), E_DEVICE, E_NOMEM. */
modap_status modap_create(int device, void *hip_stream, modap_ctx **out);

/* Release every resource of the context (synchronises its stream).  NULL is a no-op. */
void modap_destroy(modap_ctx *ctx);

/* Load the system A x <= b (section 2, eq. 1) and the starting point x0
 * (NULL = the zero vector, the start of ModAP on lists, section 3).  A is m x n in `storage`
 * with leading dimension lda; b is [m]; x0 is [n].  The library copies the data
 * into its own row-padded layout, computes ||a_i||^2 in FP64 and synchronises.
 * Resets iteration counters, the drift schedule and any pending update.
 * Errors: E_INVAL (m < 1, n < 1, lda < n, NULL A or b, non-finite b or x0,
 * bad dtype), E_ZERO_ROW (a row is zero or contains a non-finite value),
 * E_NOMEM, E_DEVICE. */
modap_status modap_set_system(modap_ctx *ctx, int64_t m, int64_t n, modap_dtype storage,
                              const void *A, int64_t lda, const double *b, const double *x0,
                              int ptrs_on_device);

/* Replace the current approximation by x ([n], NULL = zero) and reset the
 * iteration counters (checkpoint resume).  A host x must be finite (E_INVAL);
 * a device x is copied without inspection, and a non-finite entry in it stops
 * the next iterate or solve with E_NUMERIC.  Errors: E_STATE, E_INVAL. */
modap_status modap_set_x(modap_ctx *ctx, const double *x, int ptrs_on_device);

/* Update the data between iterations (the data update of ModAP on lists and of
 * ModAPL, section 3): first, k >= 0 rows are replaced in place -- row rows[q] becomes
 * new_rows[q*n .. q*n+n) (storage type, [k x n] row-major) and b[rows[q]]
 * becomes new_b[q], with ||a_i||^2 refreshed; then, when translate_v != NULL,
 * the feasible set is translated by +v: b <- b + A v.  The translation is not
 * applied by a separate pass over A: it is carried into the next sweep, which
 * reads A anyway.  Updates take effect at the next sweep in call order.  A
 * translation still pending from an earlier call or from the drift schedule
 * has already happened to the data: it does not move the new rows.  rows
 * must be distinct and in [0, m).  For host inputs a repeated or
 * out-of-range index is E_INVAL and a zero or non-finite row E_ZERO_ROW from
 * this call; for device inputs each is detected on the device before any
 * row is written, and reported as E_ZERO_ROW by the next synchronising call
 * (the context must then be loaded again).  Errors: E_STATE, E_INVAL, E_ZERO_ROW. */
modap_status modap_update_coeffs(modap_ctx *ctx, int64_t k, const int64_t *rows,
                                 const void *new_rows, const double *new_b,
                                 const double *translate_v, int ptrs_on_device);

/* Install a drift schedule for iterate/solve: after the s-th step taken from
 * now (s = 0, 1, ..., T-1) the system is translated by V[s] (row s of a
 * [T x ldv] FP64 array, ldv >= n), i.e. b <- b + A V[s], fused into the next
 * sweep.  This is the non-stationary workload of section 5 (a polytope moved
 * by a translation between iterations).  T = 0 or V = NULL removes it.
 * Errors: E_STATE, E_INVAL, E_NOMEM. */
modap_status modap_set_drift(modap_ctx *ctx, int64_t T, const double *V, int64_t ldv,
                             int ptrs_on_device);

/* Queue k >= 0 iterations (the loop of ModAP on lists, section 3, each a sweep at the
 * current x and data followed by a step, unless that sweep finds x
 * eps-feasible, after which the remaining queued iterations do nothing).
 * With out == NULL the call returns without waiting; with out != NULL it
 * synchronises and fills the statistics.  Errors: E_STATE, E_INVAL; with out
 * != NULL also E_INFEASIBLE, E_NUMERIC, E_ZERO_ROW, E_DEVICE. */
modap_status modap_iterate(modap_ctx *ctx, const modap_params *params, int64_t k,
                           modap_stats *out);

/* Iterate until x is eps-feasible (OK), max_iters steps were taken
 * (E_NOT_CONVERGED), no step direction exists (E_INFEASIBLE) or a NaN/Inf
 * appears (E_NUMERIC).  The host reads the device's stop flag once per batch
 * of queued iterations; no per-iteration synchronisation.  out may be NULL. */
modap_status modap_solve(modap_ctx *ctx, const modap_params *params, modap_stats *out);

/* One sweep at the caller's point x ([n]) on the current data (including any
 * pending update), without changing the context's state: r ([m], optional,
 * NULL to skip) = A x - b, y ([n], required) = sum of the positive slices,
 * *h = number of violated rows, *max_viol = max_i max(r_i,0)/||a_i||
 * (h and max_viol may be NULL).  x, r and y are all host or all device
 * memory according to ptrs_on_device.  Synchronises.
 * Errors: E_STATE, E_INVAL, E_DEVICE. */
modap_status modap_eval_sweep(modap_ctx *ctx, const double *x, double *r, double *y,
                              int64_t *h, double *max_viol, int ptrs_on_device);

/* Read the current approximation x ([n]) and right-hand side b ([m]) and
 * the statistics; any of x, b, out may be NULL.  b is the data as the caller
 * sees them -- every translation given so far applied, pending ones included
 * -- computed in FP64 as bref + A w (see "Exact data" above) without
 * committing anything, so reading b never changes the iteration.
 * Synchronises.  Errors: E_STATE, E_DEVICE. */
modap_status modap_query(modap_ctx *ctx, double *x, double *b, modap_stats *out,
                         int ptrs_on_device);

/* Force the sweep's kernel shape (used by the autotuner and by tests of
 * every shape); tile == NULL restores the built-in choice.  Returns E_INVAL
 * for a shape the library does not provide for the loaded system. */
modap_status modap_set_tile(modap_ctx *ctx, const modap_tile *tile);

/* The kernel shape in use for the loaded system.  Errors: E_STATE, E_INVAL. */
modap_status modap_get_tile(modap_ctx *ctx, modap_tile *tile);

/* Autotuner: time every compiled sweep shape that covers the loaded rows, at
 * one and two workgroups per CU and at full occupancy, in both row orders,
 * with `reps` stateless sweeps each, run back to back after an untimed one
 * (the context's state is not changed; the shortest counts), and return the
 * choice in *best (may be NULL).  The built-in shape is timed first and is
 * kept unless another is at least 2% faster.
 * When the environment variable MODAP_TUNE_CACHE names a file, results are
 * appended to it (one line per storage type, padded row length and m) and
 * modap_set_system uses a cached shape for the same key.  Synchronises.
 * Errors: E_STATE, E_INVAL (reps < 1), E_DEVICE. */
modap_status modap_autotune(modap_ctx *ctx, int reps, modap_tile *best);

/* ------------------------------------------------------------------------
 * Batches: many independent systems of uneven size advanced together.
 *
 * Every system of a batch is the problem above (its own data, x, drift,
 * updates, stop test and step, with the same parameters for all), and one
 * iteration of the batch is one iteration of every system that is still
 * running.  All systems of a batch share one storage type.  The sweeps of all
 * systems run in one persistent kernel launch: work items (bands of rows of
 * one system) are taken from a device queue, one wavefront per row; then one
 * launch reduces every system's y and applies its step.  Each item writes its
 * own partial sums, so a system's results are the same, bit for bit, whatever
 * other systems share the batch.  Rows are limited to 2048 (FP32), 4096
 * (BF16) or 1024 (FP64) elements; longer systems use a single-system context.
 * Conventions (ownership, ptrs_on_device, ordering, layout, precision) are
 * those of the single-system calls.
 * ------------------------------------------------------------------------ */
typedef struct modap_batch modap_batch;

typedef struct {
    int64_t iters;          /* batch iterations queued by this call */
    int64_t running;        /* systems still iterating after the call */
    int64_t systems;        /* systems in the batch */
    double seconds;         /* host wall time of this call */
    double hbm_bytes;       /* algorithmic bytes of the sweeps of this call (as in modap_stats,
                               counting every system queued) */
    double sweep_ms;        /* profile: summed duration of the batch sweep kernels */
    double reduce_ms;       /* profile: summed duration of the batch reductions */
    int64_t profiled;       /* profile: iterations timed */
} modap_batch_stats;

/* Batch tuning: target bytes of A per work item for each row-length bucket
 * (rows of at most 64*VEC*C elements, C = 1, 2, 4, 8, VEC = 16 bytes / element
 * size), the persistent grid, and the least number of items per system.  A
 * system smaller than min_items items of its bucket's size is cut into
 * min_items items of at least 32 KiB instead.  The cut of a system depends on
 * the system and this tile only, never on the other systems; a system's
 * results depend on its cut (the order in which item partials are added). */
typedef struct {
    int32_t item_kib[4];    /* largest KiB of A per work item, buckets C = 1, 2, 4, 8 (>= 1) */
    int32_t grid;           /* workgroups of the batch sweep (0: every workgroup that can be resident) */
    int32_t min_items;      /* items per system at least, 1 .. 64 (0: the library's choice, 8) */
} modap_batch_tile;

/* Create an empty batch for systems stored in `storage` on HIP device
 * `device`, queuing on hip_stream (NULL: the device's default stream).
 * Errors: E_INVAL, E_DEVICE, E_NOMEM. */
modap_status modap_batch_create(int device, void *hip_stream, modap_dtype storage, modap_batch **out);

/* Release the batch and every system in it.  NULL is a no-op. */
void modap_batch_destroy(modap_batch *batch);

/* Add the system A x <= b with starting point x0 (NULL = 0), laid out as for
 * modap_set_system; *id receives its handle.  The system joins the batch at
 * the next iteration, with fresh counters.  Synchronises.  Errors: E_INVAL
 * (sizes, NULL, lda < n, rows longer than the batched sweep covers,
 * non-finite b or x0), E_ZERO_ROW, E_NOMEM, E_DEVICE. */
modap_status modap_batch_add(modap_batch *batch, int64_t m, int64_t n, const void *A, int64_t lda,
                             const double *b, const double *x0, int ptrs_on_device, int64_t *id);

/* Remove a system from the batch and free its memory.  Errors: E_INVAL (unknown id). */
modap_status modap_batch_remove(modap_batch *batch, int64_t id);

/* Drift schedule of one system (see modap_set_drift).  Errors: E_INVAL, E_NOMEM. */
modap_status modap_batch_set_drift(modap_batch *batch, int64_t id, int64_t T, const double *V, int64_t ldv,
                                   int ptrs_on_device);

/* Data update of one system between iterations (see modap_update_coeffs).
 * Errors: E_INVAL, E_ZERO_ROW. */
modap_status modap_batch_update(modap_batch *batch, int64_t id, int64_t k, const int64_t *rows,
                                const void *new_rows, const double *new_b, const double *translate_v,
                                int ptrs_on_device);

/* Queue k iterations of every running system (see modap_iterate); out may be
 * NULL (then the call does not wait, and a stop is left for the certificate
 * of the next synchronising call, when params.certify asks for one).
 * Errors: E_STATE (empty batch), E_INVAL, E_DEVICE. */
modap_status modap_batch_iterate(modap_batch *batch, const modap_params *params, int64_t k,
                                 modap_batch_stats *out);

/* Iterate until no system is running: each stops on its own when
 * eps-feasible, after max_iters steps, without a step direction or on a
 * NaN/Inf; the per-system outcome is read with modap_batch_query.  The host
 * reads the number of running systems once per batch of queued iterations.
 * out may be NULL.  Errors: E_STATE, E_INVAL, E_DEVICE. */
modap_status modap_batch_solve(modap_batch *batch, const modap_params *params, modap_batch_stats *out);

/* Read one system's x ([n]), b ([m], pending translations applied) and
 * statistics (out->state, iters, max_viol, ...; seconds and the profile
 * fields are 0).  Any of x, b, out may be NULL.  Synchronises.
 * Errors: E_INVAL (unknown id), E_DEVICE. */
modap_status modap_batch_query(modap_batch *batch, int64_t id, double *x, double *b, modap_stats *out,
                               int ptrs_on_device);

/* Set (tile != NULL) or reset (NULL) the batch tuning, or read it (the
 * grid as requested; a launch never uses more workgroups than there are work
 * items).  Errors: E_INVAL. */
modap_status modap_batch_set_tile(modap_batch *batch, const modap_batch_tile *tile);
modap_status modap_batch_get_tile(modap_batch *batch, modap_batch_tile *tile);

/* Autotuner of the batch: for each row-length bucket present, the item size
 * (KiB of A per work item, from 64 to 16384), then the least number of items
 * per system (1 to 16) and then the grid are chosen by timing `reps`
 * stateless batch sweeps of the current systems, run back to back after an
 * untimed one (their state is not changed; the shortest counts).  A candidate
 * that cuts every system as the incumbent does is not timed, and a challenger
 * must be at least 2% faster.  The result is kept and returned in *best (may
 * be NULL); on failure the batch keeps its tile.  Synchronises.  Errors:
 * E_STATE (empty batch), E_INVAL, E_DEVICE. */
modap_status modap_batch_autotune(modap_batch *batch, int reps, modap_batch_tile *best);

/* Message describing the last failing call on the batch. */
const char *modap_batch_last_error(modap_batch *batch);

/* ------------------------------------------------------------------------
 * Solve server: continuous batching of requests on one GPU.
 *
 * Each request is a system A x <= b (storage type of the server) with a
 * starting point and an optional drift schedule, solved with the server's
 * parameters.  Requests wait in arrival order until their device footprint
 * fits the HBM budget; an admitted request whose rows fit the batched sweep
 * joins the server's batch, a larger one gets a context on its own stream,
 * so the work of all live requests overlaps on the device.  The caller drives
 * the server: each modap_server_round queues iters_per_round iterations for
 * every live request, waits for them, and retires the requests that stopped
 * (eps-feasible, no direction, NaN, or max_iters steps), freeing their device
 * memory for waiting requests.  A request's result depends only on its own
 * data, updates and rounds, not on the other requests served with it.
 * Times are seconds on the caller's clock (`now` arguments).
 * ------------------------------------------------------------------------ */
typedef struct modap_server modap_server;

typedef struct {
    int32_t state;          /* 0 queued, 1 live, 2 done, 3 failed at admission */
    int32_t status;         /* done: the system's state (1 eps-feasible, 2 no direction, 3 NaN,
                               4 step limit); failed: -modap_status */
    int32_t batched;        /* served by the batch (1) or by a context of its own (0) */
    int32_t pad;
    int64_t iters;          /* steps taken */
    int64_t sweeps;         /* checks done */
    double max_viol;        /* last check: max_i max(r_i,0)/||a_i|| */
    double eps_abs;         /* the threshold applied */
    double t_submit, t_admit, t_done;   /* caller-clock seconds (-1 = not yet) */
    double hbm_bytes;       /* algorithmic bytes of the request's sweeps */
    double footprint;       /* device bytes held while live */
} modap_request_info;

/* Create a server on `device` for systems stored in `storage`, admitting
 * requests while the sum of their footprints stays within hbm_budget_bytes.
 * params: lambda, eps, eps_relative, step and max_iters of every request.
 * Errors: E_INVAL, E_DEVICE, E_NOMEM. */
modap_status modap_server_create(int device, modap_dtype storage, double hbm_budget_bytes,
                                 const modap_params *params, int iters_per_round, modap_server **out);

/* Release the server and every request (live ones are dropped).  NULL is a no-op. */
void modap_server_destroy(modap_server *server);

/* Queue a request: A [m x n] (lda = n), b [m], x0 [n] or NULL, and a drift
 * schedule V [T x ldv] (T = 0: none).  The inputs are copied before the call
 * returns -- host inputs into host memory, device inputs into device memory
 * of the server (their producer must have finished writing them) -- so the
 * caller may release or reuse them at once.  The copy is held while the
 * request waits and released at admission; it is not counted against the
 * budget, which governs live requests.  *ticket identifies the request.
 * Errors: E_INVAL, E_NOMEM (the request alone exceeds the budget, or no
 * memory for the copy), E_DEVICE. */
modap_status modap_server_submit(modap_server *server, int64_t m, int64_t n, const void *A,
                                 const double *b, const double *x0, int64_t T, const double *V,
                                 int64_t ldv, int ptrs_on_device, double now, int64_t *ticket);

/* Data update of a live request (see modap_update_coeffs), applied before
 * its next iteration.  Device buffers are copied before the call returns
 * (their producer must have finished writing them), host buffers are read
 * during the call: either may be reused at once.  Errors: E_INVAL (unknown
 * ticket, k out of range), E_STATE (not live), E_ZERO_ROW, E_NOMEM,
 * E_DEVICE. */
modap_status modap_server_update(modap_server *server, int64_t ticket, int64_t k, const int64_t *rows,
                                 const void *new_rows, const double *new_b, const double *translate_v,
                                 int ptrs_on_device);

/* One round: admit waiting requests that fit, iterate every live request
 * iters_per_round times, wait, retire the requests that stopped.
 * *outstanding (may be NULL) receives the number of queued plus live
 * requests.  Errors: E_DEVICE and the errors of the calls it makes. */
modap_status modap_server_round(modap_server *server, double now, int64_t *outstanding);

/* Admit at most max_live requests at a time (0: no limit besides the
 * budget); 1 serves the requests one after the other.  Errors: E_INVAL. */
modap_status modap_server_set_max_live(modap_server *server, int64_t max_live);

/* Keep at most max_long requests live whose rows are too long for the
 * batched sweep (each gets a context of its own; 0, the default: no limit
 * besides the budget).  A long request beyond the limit waits in the queue,
 * and requests behind it whose rows fit the batch may be admitted past it;
 * so the long requests run with the device's bandwidth between their
 * updates instead of sharing it, while the short ones keep flowing.  A
 * request's result still depends only on its own data, updates and rounds.
 * Errors: E_INVAL. */
modap_status modap_server_set_max_long(modap_server *server, int64_t max_long);

/* State and statistics of a request.  Errors: E_INVAL. */
modap_status modap_server_info(modap_server *server, int64_t ticket, modap_request_info *out);

/* The final x ([n] host memory) of a finished request.  Errors: E_INVAL,
 * E_STATE (not finished, or its result released). */
modap_status modap_server_result(modap_server *server, int64_t ticket, double *x);

/* Free the stored result of a finished (done or failed) request.  The server
 * keeps every result until it is released or the server is destroyed, so a
 * long-running caller releases each one once it has been read.  The request's
 * statistics stay readable with modap_server_info; modap_server_result then
 * fails with E_STATE.  Releasing twice is a no-op.  Errors: E_INVAL (unknown
 * ticket), E_STATE (the request is queued or live). */
modap_status modap_server_release(modap_server *server, int64_t ticket);

/* Totals: algorithmic bytes of all sweeps so far, rounds run, device bytes
 * held by live requests (any pointer may be NULL). */
modap_status modap_server_totals(modap_server *server, double *hbm_bytes, int64_t *rounds,
                                 double *memory_in_use);

/* Message describing the last failing call on the server. */
const char *modap_server_last_error(modap_server *server);

/* One sweep with no allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid it): the pure sweep of modap_eval_sweep on a system given in
 * device memory, with no context.  A is [m x lda] device memory in `storage`
 * with lda >= n and lda a multiple of 16 bytes, columns [n, lda) zero; b [m],
 * x [n] and the outputs y [n] (required), r [m], *h and *max_viol (each may
 * be NULL) are device memory of `device`.  The work is queued on hip_stream
 * (NULL: the device's default stream) and nothing waits for it.  Every
 * intermediate lives in a 32 MiB device array of the library, one per GPU,
 * held until the process ends: calls on one GPU share it, so calls that
 * overlap on one GPU (on different streams) race.  Rows must be non-zero
 * (a zero row gives NaN, not an error).  It calls no allocator.
 * Errors: E_INVAL (sizes, NULL, lda, storage, rows too long for the one-pass
 * sweep, or a system whose norms, working vectors and partial sums exceed
 * the 32 MiB -- e.g. above about 3.5 million rows, or FP32 rows above
 * 16384 elements), E_DEVICE. */
modap_status modap_eval_sweep_static(int device, void *hip_stream, int64_t m, int64_t n, modap_dtype storage,
                                     const void *A, int64_t lda, const double *b, const double *x, double *r,
                                     double *y, int64_t *h, double *max_viol);

/* Message for a status code (static storage). */
const char *modap_strerror(modap_status status);

/* Message describing the last failing call on ctx (valid until the next call). */
const char *modap_last_error(modap_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MODAP_H */
