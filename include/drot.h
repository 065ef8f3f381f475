/*
 * drot.h -- C ABI of the MI355X (gfx950) DROT library, libdrot.so.
 *
 * DROT is Douglas-Rachford splitting applied to the discrete optimal transport
 * linear program (Mai, Lindbaeck, Johansson, "A Fast and Accurate Splitting
 * Method for Optimal Transport: Analysis and Implementation"):
 *
 *     minimise <C, X>  subject to  X 1_n = p,  X^T 1_m = q,  X >= 0     (eq. 1)
 *
 * with C (m x n) >= 0 and p, q nonnegative with equal total mass.  The library
 * runs Algorithm 1 of the paper on the GPU: one fused pass over the dense
 * m x n plan per iteration (clamped X-update with the row shift phi, the
 * column shift psi and the cost term; row sums, column sums, <C,X> and the
 * dual-residual partial in the same pass), followed by the O(m+n) shift and
 * accumulator update and the primal-dual stopping test of Section 3
 * ("Stopping criteria").
 *
 * Conventions for every entry point
 *  - All array arguments are DEVICE pointers on the context's GPU, owned by the
 *    caller (for example the storage of torch tensors).  The library never
 *    frees or keeps them beyond the documented lifetime.  `drot_result` and
 *    the host buffers of drot_get_trace are HOST memory.
 *  - Matrices are row-major: entry (i, j) of X lives at X[i * ldx + j]
 *    (row i = source i with mass p_i, column j = target j with mass q_j).
 *    Leading dimensions whose rows start on 128-byte cache lines (ld a
 *    multiple of 32 float32, 16 float64 or 64 bfloat16 elements) let the
 *    sweep read each line of X and C once; otherwise the lines shared by
 *    neighbouring column strips are fetched twice (about 10% more bytes at
 *    10000 x 15000 float32 with ld = n).
 *  - Element type: `dtype` selects float (DROT_F32) or double (DROT_F64) for
 *    C, X, p and q.  Dual outputs and warm starts (mu, nu) are always double.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *    drot_solve blocks the calling host thread until the stopping test is met
 *    (it polls a device flag every `check_every` iterations).
 *  - No exceptions cross the ABI.  Every entry point returns a drot_status;
 *    on error a message is available from drot_last_error() (thread-local).
 *    Argument errors are detected before any GPU work is enqueued; errors that
 *    need the data (unequal mass, non-finite input) are detected by the
 *    initialisation pass, before the first iteration.
 *  - A context is not thread-safe: use one context per host thread.  Calls on
 *    one context must not overlap.
 */
#ifndef DROT_H
#define DROT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct drot_ctx drot_ctx;

typedef enum {
  DROT_OK = 0,            /* stopping test met; outputs valid */
  DROT_MAXITER = 1,       /* max_iter reached first; outputs valid */
  DROT_EINVAL = -1,       /* invalid argument (size, leading dim, pointer, parameter) */
  DROT_EMASS = -2,        /* negative marginal entry or sum(p) != sum(q) */
  DROT_ENONFINITE = -3,   /* NaN/Inf in the inputs or in the iteration */
  DROT_ENOMEM = -4,       /* workspace allocation failed */
  DROT_EDEVICE = -5,      /* no usable GPU, or a HIP runtime error */
  DROT_EUNSUPPORTED = -6, /* valid but unsupported combination */
  DROT_ESTATE = -7        /* call out of order (e.g. iterate before bind) */
} drot_status;

typedef enum { DROT_F32 = 0, DROT_F64 = 1 } drot_dtype;

/* Stopping-test modes (Section 3, "Stopping criteria").  With
 *   r_primal = sqrt(|X e - p|^2 + |X^T f - q|^2),
 *   r_dual   = |[mu e^T + f nu^T - C]_+|_F,  mu = phi/rho, nu = psi/rho,
 *   gap      = |<C,X> - (p.mu + q.nu)|,
 * DROT_TOL_RELATIVE stops when max(r_primal / sqrt(|p|^2+|q|^2),
 * r_dual / |C|_F, gap / max(|<C,X>|, |p.mu+q.nu|)) <= tol, and
 * DROT_TOL_ABSOLUTE when max(r_primal, r_dual, gap) <= tol.  During the
 * iteration r_dual is the value at the shifts that entered the current
 * update (it is computed from the same read of C), one iteration behind
 * r_primal and gap; drot_finish reports all three at the returned pair. */
typedef enum { DROT_TOL_RELATIVE = 0, DROT_TOL_ABSOLUTE = 1 } drot_tol_mode;

/* Initial plan.  DROT_X0_PQ: X_0 = p q^T (the paper's experiments).
 * DROT_X0_GIVEN: X holds X_0 on entry (any nonnegative matrix). */
typedef enum { DROT_X0_PQ = 0, DROT_X0_GIVEN = 1 } drot_x0_mode;

/* How the sweep's loads and stores of X and C use the caches.  Streaming
 * (nontemporal) accesses pay off once X and C no longer fit in the 256 MB
 * last-level cache; below that, cached accesses let iterations hit in it.
 * DROT_CACHE_AUTO streams when X and C together exceed 192 MiB. */
typedef enum { DROT_CACHE_AUTO = 0, DROT_CACHE_CACHED = 1, DROT_CACHE_STREAM = 2 } drot_cache_mode;

/* drot_params.flags */
#define DROT_FLAG_NO_GRAPH 0x1    /* launch eagerly instead of replaying hipGraphs */
/* Time sweep launches with hipEvents (see drot_result).  Eager mode
 * (DROT_FLAG_NO_GRAPH): every sweep goes through hipExtLaunchKernel, whose
 * events carry the dispatch's own start and end times, so the reading is the
 * kernel's duration.  Graph mode: event-record nodes around the two sweeps in
 * the middle of every graph replay; that reading also holds the dispatch
 * latency after the start event, a few microseconds per sweep. */
#define DROT_FLAG_TIME_SWEEP 0x2
/* The skip-C schedule of the paper's Claim 1 (Section 3, "Main kernel"):
 * iterations alternate between one that reads X and C and stores
 * W = X_{k+1} - rho C, and one that reads only W and stores
 * X_{k+2} = [W + phi e^T + f psi^T]_+, so that an iteration moves 10 instead of
 * 12 bytes per float32 entry on average.  The stopping test runs after the
 * C-reading iterations only (the other one has no <C,X> and no r_dual);
 * drot_finish restores X when the run ends on a C-reading iteration. */
#define DROT_FLAG_SKIP_C 0x4
/* Float32 problems: compensated sums in the sweep (the precision variant of
 * the paper's kernel, Section 3, "Main kernel": there the row, column and
 * cost sums are plain float32 sums).  Each lane keeps Neumaier-compensated
 * float32 pairs for its row, column, <C,X> and dual-residual sums, and every
 * later combination (lanes, waves, tiles, the aux kernel) is in float64, so
 * each residual carries about one float32 rounding of its terms instead of
 * one per addition.  X stays float32.  Float64 problems ignore the flag; a
 * small float32 problem that sets it runs on sweep + aux launches (not on the
 * one-workgroup path, whose lane partials are plain float32 sums); combined
 * with DROT_FLAG_SKIP_C it gives DROT_EUNSUPPORTED; ragged widths (n not a
 * multiple of 4) use the 4-byte path. */
#define DROT_FLAG_COMPENSATED 0x8

/* Small problems take a one-workgroup path: a dense cost whose plan fits the
 * registers of one 1024-thread workgroup -- in float32 n <= 64 and m <= 512,
 * n <= 128 and m <= 256, n <= 256 and m <= 128, or n <= 512 and m <= 64; in
 * float64 half those rows -- with all sweep-schedule fields 0, cache_mode
 * AUTO, neither DROT_FLAG_SKIP_C nor DROT_FLAG_TIME_SWEEP, and in float32 not
 * DROT_FLAG_COMPENSATED.  There a single workgroup runs many whole
 * iterations per launch (the same steps, state and stopping test; each
 * lane's partial sums of at most 32 entries are in the problem's type, as in
 * the sweep, and everything after them in float64), since at these sizes two
 * launches per iteration would cost more than the memory traffic;
 * DROT_FLAG_NO_GRAPH has no effect on it.  Setting any tile field keeps a
 * small problem on the sweep + aux path.  drot_result.path reports which
 * path ran. */
typedef struct {
  double rho;          /* penalty parameter rho > 0 (the paper uses rho0/(m+n)) */
  double tol;          /* stopping tolerance >= 0; 0 runs exactly max_iter iterations */
  int64_t max_iter;    /* iteration cap >= 1 */
  int32_t tol_mode;    /* drot_tol_mode */
  int32_t x0_mode;     /* drot_x0_mode */
  int32_t check_every; /* iterations between host polls of the stop flag; 0 = 32
                          (1024 on the one-workgroup path) */
  int32_t flags;       /* DROT_FLAG_* */
  /* Sweep schedule (all 0 = automatic).  A workgroup owns a strip of
   * 64 * tile_chunks * (16 / element size) columns and the row blocks
   * g, g + tile_groups, g + 2 tile_groups, ... of tile_rows rows each. */
  int32_t tile_rows;   /* rows per row block (1..4096) */
  int32_t tile_chunks; /* 16-byte column chunks per lane (1 or 2) */
  int32_t tile_unroll; /* rows whose loads a wave keeps in flight (4 or 8) */
  int32_t cache_mode;  /* drot_cache_mode for the plan and cost streams */
  int32_t tile_groups; /* row groups (workgroups per strip); 0 = one row block per
                          workgroup when cached, two when streaming */
  int32_t reserved;    /* must be 0 */
} drot_params;

typedef struct {
  int64_t iters;          /* iterations executed (K; X holds X_K) */
  int32_t status;         /* DROT_OK or DROT_MAXITER (or the error code) */
  int32_t path;           /* how the iterations ran: 0 = sweep and aux launches
                             (always in drot_solve_batched), 1 = the one-workgroup
                             path (drot_params) */
  double objective;       /* <C, X_K>, accumulated in FP64 over the returned X */
  double dual_objective;  /* p.mu + q.nu at the returned duals */
  double r_primal, r_dual, gap;          /* exact, at the returned (X, mu, nu) */
  double eps_primal, eps_dual, eps_gap;  /* the relative forms of the three */
  double seconds_to_tol;  /* device clock, start of initialisation to the end of
                             the iteration that met the test (or the last one) */
  double seconds_total;   /* host wall clock of the call */
  double sweep_ms_total;  /* with DROT_FLAG_TIME_SWEEP: summed hipEvent time of
                             the timed sweep launches, else 0 */
  int64_t sweep_timed;    /* number of sweep launches in sweep_ms_total */
  double cost_scale;      /* DROT_COST_COORDS: the scale used (given or computed), else 0 */
} drot_result;

/* Where the sweep takes the cost c_ij from.  The paper's problem allows any
 * nonnegative m x n cost (eq. 1); its experiments use squared Euclidean
 * distances between point clouds, normalised to max 1 (Section 4).  Reading
 * fewer bytes per entry is the main lever of a bandwidth-bound sweep:
 *   DROT_COST_DENSE   C stored in the problem dtype (12 B/entry/iteration in float32)
 *   DROT_COST_BF16    C stored as bfloat16 bit patterns, float32 problems only
 *                     (10 B/entry); c_ij is the bfloat16 value widened exactly
 *   DROT_COST_COORDS  c_ij = scale * sum_d (xs_id - xt_jd)^2 evaluated in float32
 *                     from float32 coordinates, float32 problems only (8 B/entry) */
typedef enum { DROT_COST_DENSE = 0, DROT_COST_BF16 = 1, DROT_COST_COORDS = 2 } drot_cost_kind;

typedef struct {
  int32_t kind;       /* drot_cost_kind */
  int32_t dim;        /* COORDS: point dimension d, 1..3 */
  const void *data;   /* DENSE: C (problem dtype); BF16: C as uint16_t bfloat16 patterns */
  int64_t ld;         /* DENSE, BF16: leading dimension in elements, >= n */
  const float *xs;    /* COORDS: source points, m x d, row-major */
  const float *xt;    /* COORDS: target points, n x d, row-major */
  double scale;       /* COORDS: > 0 the scale; 0 = 1 / max_ij |xs_i - xt_j|^2, computed
                         on the device (reported in drot_result.cost_scale) */
} drot_cost;

/* ---- library and context -------------------------------------------- */

/* Version string, static storage. */
const char *drot_version(void);

/* Static description of a status code. */
const char *drot_strerror(int status);

/* Detail of the last error raised on the calling host thread ("" if none). */
const char *drot_last_error(void);

/* Create a context on HIP device `device` (0-based).  The context owns the
 * workspace (grown on demand, kept between solves), the pinned host mirror of
 * the device state and the captured graphs.  Returns DROT_EDEVICE when no GPU
 * is usable, DROT_ENOMEM on allocation failure. */
int drot_ctx_create(drot_ctx **ctx, int device);

/* Destroy a context and release everything it owns.  NULL is accepted. */
int drot_ctx_destroy(drot_ctx *ctx);

/* ---- one-call solve (the paper's problem statement) ------------------ */

/* Solve eq. (1) with DROT (Algorithm 1) from X_0 until the stopping test or
 * params->max_iter.
 *   m, n      problem size, m >= 1, n >= 1
 *   dtype     drot_dtype of C, X, p, q
 *   C, ldc    cost matrix, m x n, leading dimension ldc >= n, entries >= 0
 *   p, q      marginals (length m and n), >= 0, sum(p) == sum(q) within
 *             8 * machine epsilon of the dtype (relative); never renormalised
 *   X, ldx    in/out plan, m x n, ldx >= n; on return X_K (never X - rho C).
 *             Read as X_0 when params->x0_mode == DROT_X0_GIVEN.
 *   mu, nu    optional outputs (double, length m and n): mu = phi_K / rho,
 *             nu = psi_K / rho, the implicit dual variables (eq. dual:var)
 *   mu0, nu0  optional warm start (double, length m and n, both or neither):
 *             the iteration starts from the shifts phi_0 = rho mu0,
 *             psi_0 = rho nu0 instead of zero; NULL = cold start
 *   out       host result record (required)
 * C, p, q are only read; C and X must not overlap. */
int drot_solve(drot_ctx *ctx, int64_t m, int64_t n, int dtype, const void *C, int64_t ldc,
               const void *p, const void *q, const drot_params *params, void *X, int64_t ldx,
               double *mu, double *nu, const double *mu0, const double *nu0, drot_result *out,
               void *stream);

/* drot_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops that must not call hipMalloc, harnesses that
 * forbid it).  The same computation as drot_solve on the calling thread's
 * current HIP device, with no context: the workspace (state record, partial
 * sums, dual vectors, trace) is a static device array of 32 MiB that every
 * GPU the library runs on holds from its first call until the process ends,
 * and iterations are launched one by one (no graphs, no events, no streams,
 * no pinned memory are created).  The caller passes C, p, q, X, mu, nu, mu0,
 * nu0 and `out` as for drot_solve.  A problem whose workspace exceeds the
 * scratch (square problems up to about 9984 x 9984 in float32 and 9472 x
 * 9472 in float64 fit) returns DROT_EINVAL before any device work;
 * DROT_FLAG_TIME_SWEEP returns DROT_EUNSUPPORTED.  All calls on
 * one GPU share its scratch, whose contents persist between calls (every
 * call initialises what it reads): calls that overlap in time on one GPU --
 * from several host threads or streams -- race and must not be made. */
int drot_solve_noalloc(int64_t m, int64_t n, int dtype, const void *C, int64_t ldc,
                       const void *p, const void *q, const drot_params *params, void *X,
                       int64_t ldx, double *mu, double *nu, const double *mu0,
                       const double *nu0, drot_result *out, void *stream);

/* ---- step-wise interface (same computation, split at its natural seams) -- */

/* Bind a problem to the context and run the initialisation of Algorithm 1
 * (X_0, phi_0, psi_0, a_0, b_0, alpha_0) plus the scale factors of the
 * relative stopping test.  Arguments as for drot_solve.  The pointers must
 * stay valid until the next bind or the context's destruction.  Blocks until
 * the initialisation pass has validated the data. */
int drot_bind(drot_ctx *ctx, int64_t m, int64_t n, int dtype, const void *C, int64_t ldc,
              const void *p, const void *q, const drot_params *params, void *X, int64_t ldx,
              const double *mu0, const double *nu0, void *stream);

/* Enqueue `iters` further iterations of Algorithm 1 (one sweep and one dual
 * update each; on the one-workgroup path, launches of up to 4096 whole
 * iterations) on `stream` without waiting.  Iterations after the stopping
 * test (or max_iter) has fired are no-ops on the device. */
int drot_iterate(drot_ctx *ctx, int64_t iters, void *stream);

/* Autotune the tile variant of the sweep for the bound problem.  Not an
 * operation of the paper: the sweep of Algorithm 1 (Section 3) can be tiled
 * many ways, and which is fastest depends on the shape.  Each candidate --
 * rows per block in {8, 16, 32} x {1, 2} 16-byte chunks per lane (on the
 * scalar path 1 or 4 elements) x one or two row blocks per workgroup, with
 * the bound cache_mode -- is bound (initialisation included), warmed up for
 * one graph and timed over `iters` iterations (0 = four graphs; rounded up to
 * whole graphs) with hipEvents on `stream`.  The fastest is then bound again
 * with the caller's other parameters, ready for drot_iterate from iteration
 * 0, and returned in *best (host; tile_rows, tile_chunks and tile_groups set).
 * *us_per_iter (host, may be NULL) receives its time per iteration.  A
 * problem on the one-workgroup path (drot_params) has no tile variants: it is
 * timed as bound (`iters` iterations, 0 = 256), bound again, and *best is the
 * caller's parameters.  X is overwritten by the trials, so the problem must have been bound with
 * x0_mode = DROT_X0_PQ (else DROT_EUNSUPPORTED); DROT_ESTATE without a bound
 * problem.  Blocks until done. */
int drot_tune(drot_ctx *ctx, int64_t iters, drot_params *best, double *us_per_iter,
              void *stream);

/* Wait for `stream` and report progress: iterations done so far and whether
 * the stop flag is set (1) or not (0). */
int drot_poll(drot_ctx *ctx, int64_t *iters_done, int32_t *stopped, void *stream);

/* Final evaluation pass: exact residuals, objectives and gap of the current
 * (X, mu, nu), accumulated in FP64; writes mu and nu if non-NULL and fills
 * `out`.  Blocks until done. */
int drot_finish(drot_ctx *ctx, double *mu, double *nu, drot_result *out, void *stream);

/* drot_bind / drot_solve with a cost descriptor instead of a dense C
 * (arguments otherwise as above).  The skip-C schedule needs a dense C. */
int drot_bind_cost(drot_ctx *ctx, int64_t m, int64_t n, int dtype, const drot_cost *cost,
                   const void *p, const void *q, const drot_params *params, void *X,
                   int64_t ldx, const double *mu0, const double *nu0, void *stream);

int drot_solve_cost(drot_ctx *ctx, int64_t m, int64_t n, int dtype, const drot_cost *cost,
                    const void *p, const void *q, const drot_params *params, void *X,
                    int64_t ldx, double *mu, double *nu, const double *mu0, const double *nu0,
                    drot_result *out, void *stream);

/* ---- many independent problems at once ------------------------------ */

/* One problem of a batch: dense cost, in the batch's dtype.  Arrays are
 * device pointers owned by the caller; mu and nu are optional outputs. */
typedef struct {
  int64_t m, n;
  const void *C;
  int64_t ldc;
  const void *p, *q;
  void *X;            /* out: X_K of this problem (X_0 = p q^T) */
  int64_t ldx;
  double rho, tol;    /* per-problem penalty and tolerance */
  double *mu, *nu;    /* out (nullable): double, length m and n */
  const double *mu0, *nu0;  /* warm start (nullable, both or neither), as in drot_solve */
} drot_problem;

/* Solve `count` independent problems of any shapes together: every iteration
 * is one batched sweep launch, one batched aux launch over the (problem, work
 * item) pairs of the problems still running and one finishing launch (one
 * wave per problem), replayed as hipGraphs of
 * params->check_every iterations.  Each problem runs Algorithm 1 with its own
 * stopping test and stops on its own; finished problems leave the work lists
 * when they make up half of them.  params supplies max_iter, tol_mode,
 * check_every, cache_mode, tile_rows, tile_chunks, tile_groups and
 * DROT_FLAG_NO_GRAPH; each problem's sweep schedule (rows per block, blocks
 * per work item) comes from the context's tuner cache for its size class
 * (drot_tune_batched) unless tile_rows / tile_groups set it.  outs[count] receives one result per
 * problem.  Returns DROT_OK when every problem met its test, DROT_MAXITER if
 * some hit max_iter, or an error (the message names the problem).  The call
 * uses the context's workspace and releases a problem bound by drot_bind. */
int drot_solve_batched(drot_ctx *ctx, int32_t count, int dtype, const drot_problem *probs,
                       const drot_params *params, drot_result *outs, void *stream);

/* Autotuner of the batched sweep's schedule.  Not an operation of the paper:
 * a batch mixes problems of very different shapes, and the shape of a sweep
 * work item -- 16-byte chunks per lane (the strip width), rows per block and
 * row blocks per item -- decides how long each workgroup lives and how many
 * column partials the aux kernel adds.  Problems are grouped by size class
 * of (m, n), each side in one of [1,128), [128,256), [256,512), [512,1024),
 * [1024,2048), [2048,inf).  Stage 1 times the whole batch under one schedule
 * for every class: chunks in {1, 2} x rows in {8, 16, 32} x blocks per item
 * in {1, 2}.  Stage 2 revisits each class holding at least 5% of the
 * entries, largest first, with rows in {8, 16, 32} x blocks in {1, 2, 4}
 * while the other classes keep theirs, and keeps a change that is 1%
 * faster.  Each timing is `iters` iterations of the whole batch (0 = two
 * graphs of params->check_every; rounded up to whole graphs) after one warm
 * graph, under the batch's cache policy.  The choices go to the context's
 * tuner cache, which drot_solve_batched consults (untuned: 2 chunks, 16-row
 * blocks, one per item; params->tile_chunks, tile_rows and tile_groups, when
 * set, override).  `table` (host, table_cap entries, may be NULL if
 * table_cap is 0) receives one entry per class present and *n_entries their
 * number.  The problems' X arrays are overwritten by the trials.  Blocks
 * until done. */
typedef struct {
  int32_t m_class, n_class;   /* size classes 0..5 of m and n (see above) */
  int32_t tile_rows;          /* chosen rows per block */
  int32_t blocks_per_item;    /* chosen row blocks per sweep work item */
  int32_t problems;           /* problems of the class in the batch */
  int32_t chunks;             /* chosen 16-byte chunks per lane (whole batch) */
  double us_per_iter;         /* the whole batch per iteration with the final choices */
} drot_batch_tile;

int drot_tune_batched(drot_ctx *ctx, int32_t count, int dtype, const drot_problem *probs,
                      const drot_params *params, int64_t iters, drot_batch_tile *table,
                      int32_t table_cap, int32_t *n_entries, void *stream);

/* ---- learned warm start: a small MLP trained with this library's kernels ---
 * Not part of the paper: a network maps (p, q) to initial dual variables
 * (mu, nu); DROT then starts from phi_0 = rho mu, psi_0 = rho nu (drot_solve's
 * mu0/nu0), which is valid because DR converges from any start (Lemma 1).
 * Architecture in -> hidden (ReLU) -> hidden (ReLU) -> out, mean-squared
 * error.  Float32 master weights and Adam; bfloat16 copies feed the matrix
 * cores (32x32x8 bfloat16 MFMA, float32 accumulation).  Widths and batches
 * are multiples of 64.  The flat parameter vector is [W1, b1, W2, b2, W3, b3]
 * with W_l stored row-major as out_l x in_l.  x, y, t and grad are device
 * float32 arrays, row-major batch x width.  The network owns its device
 * buffers (parameters, Adam moments, activations for max_batch rows and a
 * 4 MiB split-K workspace) and reuses them on every call: calls on one
 * network must be ordered (one stream, or synchronised), not concurrent. */
typedef struct drot_mlp drot_mlp;
int drot_mlp_create(drot_mlp **mlp, int device, int in_dim, int hidden, int out_dim,
                    int max_batch, uint64_t seed);
int drot_mlp_destroy(drot_mlp *mlp);
int drot_mlp_num_params(const drot_mlp *mlp, int64_t *count);
int drot_mlp_set_weights(drot_mlp *mlp, const float *host);  /* also resets Adam */
int drot_mlp_get_weights(drot_mlp *mlp, float *host);
int drot_mlp_forward(drot_mlp *mlp, int batch, const float *x, float *y, void *stream);
/* Loss (host, FP64-accumulated mean squared error) and its gradient w.r.t.
 * the flat parameters (grad may be NULL). */
int drot_mlp_gradients(drot_mlp *mlp, int batch, const float *x, const float *t, float *grad,
                       double *loss, void *stream);
/* One Adam step (Kingma and Ba, 2015: beta1 0.9, beta2 0.999, eps 1e-8, bias
 * corrections 1 - beta^k at the network's k-th step) on the batch's loss. */
int drot_mlp_train_step(drot_mlp *mlp, int batch, const float *x, const float *t, float lr,
                        double *loss, void *stream);
/* The same Adam step with a caller-supplied gradient `grad` (device float32,
 * the flat parameter order, n_params entries; only read), e.g. gradients
 * summed over several data-parallel replicas before the step.  Shares the
 * step counter and moment estimates with drot_mlp_train_step.  lr > 0 and
 * grad != NULL, else DROT_EINVAL. */
int drot_mlp_apply_gradients(drot_mlp *mlp, const float *grad, float lr, void *stream);

/* ---- checkpoint and resume (not in the paper; the iteration state of
 * Algorithm 1 is X plus the O(m+n) vectors and scalars listed there) ------- */

/* Size in bytes of a checkpoint of the bound problem. */
int drot_checkpoint_size(drot_ctx *ctx, size_t *bytes);

/* Copy the iteration state of the bound problem -- the device state record
 * (iteration count, alpha, the scalar shift parts, stopping-test scale
 * factors), a, b, phi, psi and the trace -- to `host_buf` (host memory, at
 * least drot_checkpoint_size bytes, owned by the caller) after the work
 * enqueued on `stream` has finished.  X is the caller's array and is not
 * copied: save it alongside.  Under DROT_FLAG_SKIP_C only after an even
 * number of iterations (else X holds X - rho C: DROT_ESTATE). */
int drot_checkpoint(drot_ctx *ctx, void *host_buf, size_t bytes, void *stream);

/* Continue a checkpointed run: bind the same problem first (same m, n,
 * dtype, cost kind and skip-C flag; X holding the checkpointed plan and
 * x0_mode = DROT_X0_GIVEN, so that the initialisation pass only validates
 * it), then call drot_resume.  The next drot_iterate continues from the
 * checkpointed iteration with the bound tol, tol_mode and max_iter (which
 * counts all iterations, before and after the checkpoint); device times are
 * measured from the resume.  A mismatched or corrupt checkpoint gives
 * DROT_EINVAL and leaves the bound state as the bind made it. */
int drot_resume(drot_ctx *ctx, const void *host_buf, size_t bytes, void *stream);

/* Copy per-iteration records of the last bound problem to host memory.
 * Record k (1-based iteration index) holds 8 doubles:
 *   pobj, dobj, r_primal, r_dual (lagged, see drot_tol_mode), gap,
 *   test value (the quantity compared with tol), device seconds since the
 *   start of initialisation, k.
 * Only the last `trace capacity` iterations are kept (65536); asking for an
 * older or a future record returns DROT_EINVAL. */
int drot_get_trace(drot_ctx *ctx, int64_t first, int64_t count, double *host_out);

#ifdef __cplusplus
}
#endif

#endif /* DROT_H */
