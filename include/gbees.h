/*
 * gbees.h -- C ABI of the GBEES hot path on MI355X (gfx950).
 *
 * GBEES (Grid-based Bayesian Estimation Exploiting Sparsity, GBEES-GPU,
 * arXiv 2508.13986) propagates a probability density p(x, t), x in R^n, on a
 * sparse grid of control volumes (Sec. 2.1, Eq. 5) with the conservative
 * advection equation (Sec. 2, Eq. 3), and corrects it with Bayes' rule at
 * measurement times (Eq. 4).  One time step is: grow the grid downwind of the
 * cells above the probability threshold (Sec. 3.3), take the CFL time step
 * (Sec. 3.2, Eq. 8), compute Donor Cell Upwind fluxes (Eq. 7) with Corner
 * Transport Upwind corrections (Algorithm 1) and an optional high-resolution
 * term, update the densities, and every few steps prune cells below the
 * threshold that have no upwind neighbour above it (Algorithm 3), then
 * renormalise.
 *
 * Conventions of every entry point:
 *  - Return 0 (GBEES_OK) or a negative GBEES_E_* code (gbees_strerror names it).
 *  - Memory: the caller owns the arena, a device buffer of at least
 *    gbees_arena_bytes(cfg) bytes that must outlive the context; the library
 *    allocates no device memory.  Host buffers belong to the caller.
 *  - Streams: all device work is enqueued on the caller's HIP stream (passed
 *    as void*, may be NULL for the null stream).  Calls that return host data
 *    synchronise that stream.
 *  - Cell indices: cell i in Z^n has centre mean + i*h (mean and h from the
 *    config); index arrays are row-major [count][n] int32.
 *  - Densities are cell averages normalised so that prod(h) * sum P = 1.
 *  - Exported cells are sorted lexicographically by index.
 *  - GBEES_E_CAPACITY or GBEES_E_RANGE from gbees_step (a grow that needed
 *    more bricks or hashtable slots than max_cells provides, or a cell index
 *    outside the packable range) leaves the grid as it was at the start of the
 *    step that failed: time, step count, cells and densities.  The context
 *    stays usable: gbees_export it, or move it into a larger arena with
 *    gbees_resize and step on.  Stepping again without more capacity fails
 *    at the same step.
 *  - After any other error the context is unusable except for
 *    gbees_get_stats and gbees_destroy (every other call returns
 *    GBEES_E_STATE).
 *  - Not thread-safe per context; distinct contexts are independent.
 */
#ifndef GBEES_H
#define GBEES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GBEES_OK = 0,
  GBEES_E_ARG = -1,      /* invalid argument or configuration */
  GBEES_E_CAPACITY = -2, /* the grid outgrew max_cells (or the hashtable) */
  GBEES_E_RANGE = -3,    /* a cell index left the packable coordinate range */
  GBEES_E_DEVICE = -4,   /* a HIP runtime call failed */
  GBEES_E_BUFFER = -5,   /* output buffer too small; *count_out holds the size needed */
  GBEES_E_STATE = -6     /* the context is in an error state */
};

/* Drift models f(x).  Lorenz '63 and Lorenz '96 are the paper's test systems
 * (Sec. 5.1.1, 5.1.2); LINEAR (f = A x + b) and UNIFORM (f = b) serve tests. */
enum { GBEES_L63 = 1, GBEES_L96 = 2, GBEES_LINEAR = 3, GBEES_UNIFORM = 4 };

typedef struct gbees_ctx gbees_ctx;

typedef struct {
  int32_t n;           /* dimension: 3 for L63, 4..6 for L96, 1..6 for LINEAR/UNIFORM */
  int32_t model;       /* GBEES_L63 | GBEES_L96 | GBEES_LINEAR | GBEES_UNIFORM */
  double params[48];   /* L63: sigma, rho, beta, z_shift (f evaluated at x3 + z_shift);
                          L96: F; LINEAR: A (n*n, row-major) then b (n); UNIFORM: b (n) */
  double h[6];         /* cell widths h_j > 0 (Eq. 5) */
  double mean[6];      /* initial mean; also the centre of cell 0 */
  double cov[36];      /* initial covariance, n*n row-major, symmetric positive definite */
  double thresh_rel;   /* p* = thresh_rel * max P; 0 = grow from every non-zero cell, never prune */
  double cfl;          /* Courant number C in (0, 1]: dt = C / max_i sum_j |f_j| / h_j */
  double dt_fixed;     /* > 0 replaces the CFL step (tests) */
  int32_t prune_every; /* prune after every prune_every-th step; 0 = never */
  int32_t limiter;     /* 0: Eq. 7 + Algorithm 1 only; 1: plus the MC-limited high-resolution term */
  int32_t grow_mode;   /* 0: downwind axis and pairwise-edge neighbours; 1: every one of them;
                          2: every combination of downwind steps, one per dimension (the orthant,
                          up to 2^n - 1 cells, Sec. 3.3); prune mirrors the choice upwind.
                          The serving pool takes modes 0 and 1 only. */
  int32_t precision;   /* 0: FP64 densities; 1: FP32 densities and fluxes, FP64 reductions */
  int64_t max_cells;   /* capacity in cell slots (cells are stored in bricks of 64) */
  double hash_load;    /* hashtable load bound (Sec. 4.2), 0 => 0.5 */
} gbees_config;

typedef struct {
  double t;              /* current time */
  double dt_last;        /* last time step */
  double mass;           /* prod(h) * sum P after the last reduction */
  double max_p;          /* max P of the current grid */
  double smax;           /* max_i sum_j |f_{i-1/2 e_j, j}| / h_j over the grid */
  int64_t steps;         /* time steps taken since initialisation */
  int64_t cell_updates;  /* sum over steps of the number of cells updated */
  int64_t brick_updates; /* sum over steps of the number of bricks swept by the flux passes */
  int64_t cells;         /* cells in the grid */
  int64_t bricks;        /* bricks in use */
  int64_t prunes;        /* prune passes run */
  int64_t grow_bricks;   /* bricks the grow pass expanded (cells newly above threshold since the last prune) */
  int64_t inserted;      /* cells created by grow */
  int64_t deferred;      /* grow inserts whose brick another wave was still creating, finished by the fix-up pass */
  double mass_pruned;    /* sum over prunes of the fraction of the mass present that each prune removed */
} gbees_stats;

/* Device bytes the arena must hold for cfg (0 if cfg is invalid). */
size_t gbees_arena_bytes(const gbees_config* cfg);

/* Initial condition (Sec. 5.1: a Gaussian pdf): the grid is every cell i whose
 * centre offset y = i*h satisfies y' cov^-1 y <= 2 ln(1/thresh_rel), with
 * P = exp(-y' cov^-1 y / 2), normalised.  Requires 0 < thresh_rel < 1.
 * On success *out owns nothing but host bookkeeping; the grid lives in arena. */
int gbees_init_gaussian(const gbees_config* cfg, void* arena, size_t arena_bytes, void* hip_stream,
                        gbees_ctx** out);

/* Initial condition from caller cells: count cells with indices idx[count][n]
 * (distinct) and densities P[count] (used as given, not normalised), at time t0. */
int gbees_init_cells(const gbees_config* cfg, const int32_t* idx, const double* P, int64_t count, double t0,
                     void* arena, size_t arena_bytes, void* hip_stream, gbees_ctx** out);

/* Advance until t == t_stop exactly (the last step is clamped, Sec. 3.2), or
 * until max_steps (> 0) steps were taken.  Each step: grow, CFL step, DCU +
 * CTU fluxes (+ high-resolution term), update; prune + renormalise after every
 * prune_every-th step.  Fills *out (may be NULL). */
int gbees_step(gbees_ctx* ctx, double t_stop, int64_t max_steps, gbees_stats* out);

/* Bayesian correction (Eq. 4) with measurement y = x_component + noise,
 * noise ~ N(0, sigma^2): P_i *= exp(-(y - x_i,component)^2 / (2 sigma^2)) at
 * the cell centres, then prune (if pruning is enabled) and renormalise. */
int gbees_correct(gbees_ctx* ctx, int32_t component, double y, double sigma);

/* Marginal over the dimensions in dim_mask (bit j = keep x_j; Sec. 5.1.2):
 * M(k) = sum over cells i with i restricted to the mask equal to k of
 * P_i * prod_{j not in mask} h_j.  Writes count rows, sorted by k, into
 * idx_out[count][popcount(mask)] and val_out[count]; GBEES_E_BUFFER (with
 * *count_out set) if capacity < count. */
int gbees_marginals(gbees_ctx* ctx, uint32_t dim_mask, int64_t capacity, int32_t* idx_out, double* val_out,
                    int64_t* count_out);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid allocation): the marginal of gbees_marginals,
 * written into caller DEVICE buffers idx_dev[capacity][popcount(mask)] and
 * val_dev[capacity], rows in no particular order, with the row count stored
 * to *count_dev (device int64; -1 if the aggregation table overflowed; rows
 * past capacity are counted but not written).  Only enqueues work on the
 * context's stream: no allocation, no host copy, no wait.  The aggregation
 * table is one file-scope device array of 2^20 slots (16 MiB) per GPU, held
 * until the process ends and cleared by every call: calls that overlap on one
 * GPU (any contexts, any streams) race for it.  GBEES_E_CAPACITY for grids of
 * more than 2^19 cells.  Sums are FP64 atomics, so the last bits of a value
 * may differ between calls. */
int gbees_marginals_noalloc(gbees_ctx* ctx, uint32_t dim_mask, int64_t capacity, int32_t* idx_dev, double* val_dev,
                            int64_t* count_dev);

/* Copy the grid out: idx[count][n], P[count] sorted by index, and the time.
 * GBEES_E_BUFFER (with *count set) if capacity < count.  t may be NULL. */
int gbees_export(gbees_ctx* ctx, int64_t capacity, int32_t* idx, double* P, int64_t* count, double* t);

/* Move the grid into a new arena of at least gbees_arena_bytes(cfg with
 * max_cells) bytes, which must not overlap the current one, and keep
 * stepping there with capacity max_cells (Sec. 4.1: the capacity is fixed per
 * arena, so a grid that outgrows it moves).  Cells, densities, time, step
 * count and statistics carry over; the old arena is free for the caller once
 * this returns.  GBEES_E_CAPACITY if max_cells cannot hold the current
 * bricks.  Device-to-device copies on the context's stream; no allocation. */
int gbees_resize(gbees_ctx* ctx, int64_t max_cells, void* arena, size_t arena_bytes);

/* Current statistics (synchronises the stream). */
int gbees_get_stats(gbees_ctx* ctx, gbees_stats* out);

/* Hashtable probe lengths (Sec. 4.2): mean probes of a successful lookup of
 * every brick key, of an unsuccessful lookup of n_miss keys that are not in
 * the table, and the load factor. */
int gbees_probe_stats(gbees_ctx* ctx, int64_t n_miss, double* mean_hit, double* mean_miss, double* load);

/* Per-pass device time: when enabled, every launch of the grow, flux-A
 * (transverse-corrected states), flux-B (fluxes + update) and prune passes is
 * bracketed by HIP events on the context stream; gbees_profile_read returns
 * accumulated milliseconds and launch counts in the order grow, grow-fix,
 * flux-A, flux-B, prune, other (6 entries each) and resets them. */
int gbees_profile(gbees_ctx* ctx, int enable);
int gbees_profile_read(gbees_ctx* ctx, double* ms, int64_t* launches);

/* Release host bookkeeping (the arena stays the caller's). */
int gbees_destroy(gbees_ctx* ctx);

const char* gbees_strerror(int code);

/* ------------------------------------------------------------------------
 * Serving pool: propagation requests for many objects (each a Gaussian prior,
 * a horizon and scalar measurements: the problem of Sec. 2 and 5.1 posed per
 * object) share one caller-owned device arena.  A request is admitted when a
 * slot is free and a slice of the arena of gbees_arena_bytes(cfg) bytes can be
 * carved out (so cfg->max_cells sets its footprint).  Running requests of one
 * kind (model, dimension, precision) are stepped together, one launch per
 * kernel for all of them, by that kind's driver thread; each keeps its own
 * device state and gets the result it would get alone, up to the rounding of
 * its sums (a pooled grid's launches take more bricks per wave than a grid
 * stepped alone, since the pool's grids share the device).
 * Requests leave the pool as soon as they finish, which frees their slot for
 * the next ones (and their slice once the result was taken).  The pool
 * allocates no device memory; it owns a HIP stream per group of requests and
 * one per admitted request.  Times are seconds on the pool's monotonic
 * clock.
 * ---------------------------------------------------------------------- */
typedef struct gbees_pool gbees_pool;

typedef struct {
  double t;          /* measurement time in [0, t_end] (later ones are ignored) */
  int32_t component; /* measured coordinate, 0-based */
  double y;          /* measured value */
  double sigma;      /* noise standard deviation > 0 (Eq. 4 with a Gaussian likelihood) */
} gbees_meas;

typedef struct {
  int32_t status;      /* 0 waiting, 1 running, 2 done, < 0 the GBEES_E_* code it failed with */
  double t_submit;     /* when gbees_pool_submit accepted it */
  double t_admit;      /* when it got its slot and arena slice */
  double t_done;       /* when its last batch finished on the device (or it failed) */
  int64_t arena_bytes; /* its footprint */
  int64_t cells;       /* cells in the result */
  gbees_stats stats;   /* statistics of the finished propagation */
  int64_t resizes;     /* times the request's grid outgrew its capacity and moved into a larger slice */
} gbees_req_info;

/* arena: device buffer of arena_bytes owned by the caller for the pool's
 * life; max_active (1..256): requests running at once.  All pool calls may come
 * from any thread.  Concurrent gbees_pool_result calls for one request share
 * its one copy; gbees_pool_release during such a copy returns GBEES_E_STATE. */
int gbees_pool_create(void* arena, size_t arena_bytes, int32_t max_active, gbees_pool** out);

/* Queue a request: initialise from the Gaussian of cfg (as gbees_init_gaussian),
 * step to each measurement time in order, correct (as gbees_correct), step to
 * t_end.  Requires cfg->thresh_rel > 0.  meas is copied.  *req receives its id.
 * GBEES_E_CAPACITY if its footprint exceeds the whole arena.  A request whose
 * grid outgrows its capacity continues from the step that failed in a slice
 * of four (else two) times the capacity (gbees_resize); only when no such
 * slice is free does it end with status GBEES_E_CAPACITY. */
int gbees_pool_submit(gbees_pool* pool, const gbees_config* cfg, double t_end, const gbees_meas* meas,
                      int32_t n_meas, int64_t* req);

/* Admit waiting requests in arrival order (looking up to three places past one
 * that does not fit) to free slots and arena slices, without waiting on the
 * device; the drivers run them.  Either count may be NULL. */
int gbees_pool_progress(gbees_pool* pool, int32_t* n_running, int32_t* n_waiting);

int gbees_pool_info(gbees_pool* pool, int64_t req, gbees_req_info* out);

/* The finished request's grid, as gbees_export: idx[count][n], P[count] sorted
 * by index.  A finished request keeps its grid (and arena slice) on the device
 * until the first call of this function copies it to the host and frees the
 * slice.  GBEES_E_STATE while it runs; its error code if it failed;
 * GBEES_E_BUFFER (with *count set) if capacity < count. */
int gbees_pool_result(gbees_pool* pool, int64_t req, int64_t capacity, int32_t* idx, double* P, int64_t* count);

/* Requests of one kind that one driver steps with shared launches (1..64,
 * default 4); applies to groups formed after the call. */
int gbees_pool_group_size(gbees_pool* pool, int32_t k);

/* Forget a finished or failed request, freeing its arena slice if it still
 * holds one.  Release every finished request: its slice is not reused before. */
int gbees_pool_release(gbees_pool* pool, int64_t req);

/* Seconds on the pool's clock (0 for a NULL pool). */
double gbees_pool_clock(gbees_pool* pool);

/* Wait for the pool's streams and release everything but the arena. */
int gbees_pool_destroy(gbees_pool* pool);

#ifdef __cplusplus
}
#endif

#endif /* GBEES_H */
