/*
 * bsde.h -- C ABI of the MI355X (gfx950) BSDE solver library (libbsde.so).
 *
 * The library computes the Picard iteration with an adaptive Monte Carlo
 * control variate of Labart & Lelong, "A Parallel Algorithm for solving
 * BSDEs -- Application to the pricing and hedging of American options"
 * (arXiv:1102.4666): Algorithm 1 of Section 3.1 in the detailed form of
 * Algorithm "algodetail" (Section 4.1), applied to the option model of
 * Section 5 (log-prices, eq. 4; penalised BSDE, eq. bsde-penal-2) with the
 * correlated Brownian motion of Section 6.2.  Every step of a solve runs in
 * hand-written HIP kernels on the GPU; the host only prepares the fixed
 * grid and the least-squares factorisation once per problem.
 *
 * Conventions for every entry point:
 *  - plain C types; pointers are HOST pointers unless stated otherwise;
 *  - inputs are copied, the caller keeps ownership of its arrays;
 *  - outputs go to caller-allocated buffers of the documented size;
 *  - every call returns a bsde_status and never aborts; on error nothing
 *    is written to the outputs;
 *  - a problem handle is not thread-safe; distinct handles are independent.
 */
#ifndef BSDE_H
#define BSDE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bsde_problem_s *bsde_problem; /* owned by the library */

typedef enum {
    BSDE_OK = 0,
    BSDE_EINVAL = 1,   /* an argument is out of range                       */
    BSDE_ENOMEM = 2,   /* host or device allocation failed                  */
    BSDE_ERANK = 3,    /* fewer points than basis functions, or the basis
                          matrix is numerically rank deficient             */
    BSDE_EDEVICE = 4,  /* a HIP call failed (no GPU, launch failure, ...)    */
    BSDE_ESTATE = 5,   /* call not valid in the current state (e.g. query
                          before solve)                                    */
    BSDE_EUNSUPPORTED = 6, /* no kernel is built for this (d, eta, precision,
                              volatility kind), or a feature the entry point
                              does not serve                                */
    BSDE_EBUSY = 7     /* request not finished yet (non-blocking poll)      */
} bsde_status;

/* Volatility sigma_j(t, S) of asset j (eq. 4 of Section 5, diagonal form:
 * the diffusion of X_j is sigma_j (L dW)_j with L the Cholesky factor of the
 * correlation matrix). */
typedef enum {
    BSDE_VOL_CONST = 0, /* sigma_j = level_j                               */
    BSDE_VOL_BUMP = 1,  /* sigma_j = level_j (1 + bump_a e^{-(log(S/bump_c))^2}) */
    BSDE_VOL_DUPIRE = 2 /* eq. vol_locale: sigma(t, S) = 0.6 (1.2 -
                           e^{-0.1 t} e^{-0.001 (S e^{r t} - s)^2})
                           e^{-0.05 sqrt t}, s = S0_j (smile bottom at the
                           forward); level_j then only sets the width of D.
                           Kernels: d=1 eta=4, d=2 eta=3, d=5 eta=2,3.      */
} bsde_vol_kind;

typedef struct {
    int kind;               /* bsde_vol_kind                                 */
    const double *level;    /* d levels, > 0                                 */
    double bump_a;          /* bump height (BSDE_VOL_BUMP)                   */
    double bump_c;          /* bump centre in price units (> 0)              */
    double rho;             /* uniform correlation (Section 6.2), must lie in
                               (-1/(d-1), 1) so that rho 11' + (1-rho) I is
                               positive definite                            */
    const double *dividend; /* d dividend rates delta_j, or NULL for zeros   */
} bsde_sigma;

/* Payoff Phi of the log-price x (eqs. put_payoff, call_payoff). */
typedef enum {
    BSDE_PUT_ARITH = 0,  /* (K - (1/d) sum_j e^{x_j})_+                     */
    BSDE_CALL_ARITH = 1, /* ((1/d) sum_j e^{x_j} - K)_+                     */
    BSDE_PUT_GEOM = 2,   /* (K - exp((1/d) sum_j x_j))_+                    */
    BSDE_CALL_GEOM = 3,  /* (exp((1/d) sum_j x_j) - K)_+                    */
    BSDE_FWD_ARITH = 4,  /* (1/d) sum_j e^{x_j} - K  (call minus put)       */
    BSDE_QUAD = 5        /* (sum_j x_j)^2 (test payoff with a polynomial
                            solution when r = 0)                           */
} bsde_payoff_kind;

typedef struct {
    int kind;          /* bsde_payoff_kind                                   */
    double K;          /* strike                                             */
    double T;          /* maturity (> 0)                                     */
    const double *S0;  /* d spot prices (> 0); centre of the domain D        */
} bsde_payoff;

/* The n points (t_i, x_i) of Algorithm "algodetail" and the basis of the
 * least-squares extrapolating operator (Section 4.2, eqs. lspb and
 * hyper_set).  Points are fixed for all iterations.  Point i is
 * a * n_spatial + b for time node a (t_a = a T / (n_t - 1)) and spatial
 * point b.  The domain is D_j = log S0_j +- width * level_j * sqrt(T);
 * polynomials are Chebyshev in the variables mapped to [-1, 1]^{d+1}. */
typedef enum {
    BSDE_GRID_TENSOR = 0, /* n_x equispaced nodes per asset (endpoints
                             included); spatial point b has base-n_x digits
                             b_j, asset 1 least significant               */
    BSDE_GRID_RANDOM = 1, /* n_x points uniform in D from the counter-based
                             generator (substream 2): drawn once, or at
                             every Picard iteration with redraw            */
    BSDE_GRID_UNIFORM = 2 /* n = n_x points (t, x) uniform over [0, T] x D,
                             Algorithm 1's draw (substream 3; n_t unused),
                             once or at every iteration with redraw        */
} bsde_grid_kind;

typedef struct {
    int kind;      /* bsde_grid_kind                                        */
    int n_t;       /* time nodes, >= 2 (tensor and random kinds)            */
    int n_x;       /* tensor: nodes per asset; random: spatial points;
                      uniform: points                                      */
    double width;  /* half-width of D in units of level_j sqrt(T), > 0      */
    int eta;       /* maximal total degree of the polynomial basis          */
    double q;      /* hyperbolic index set parameter in (0, 1]; 1 = total
                      degree                                               */
    int redraw;    /* 1: random or uniform points only -- new points at
                      every Picard iteration k (Algorithm 1 draws new points
                      each iteration; counter word 2 = k, iteration 0 = the
                      fixed set), the least-squares factorisation redone
                      on the device for each; bsde_solve only (the batched
                      entry points and the server return
                      BSDE_EUNSUPPORTED).  0: one fixed grid.             */
    double kernel_bw; /* > 0: extrapolate with the kernel operator of
                      Section 3.2 (the first version of the method) instead
                      of least squares on the basis: u^{k+1}(t, x) =
                      sum_i y_i w_i / sum_i w_i over the points, y_i =
                      u^k(t_i, x_i) + c^k_i, w_i = exp(-min(|z - z_i|^2 /
                      (2 kernel_bw^2), 60)) in the coordinates z in
                      [-1, 1]^{d+1} that map [0, T] x D (the bandwidth is in
                      those units).  Supported for d <= 2, constant or bump
                      volatility, fixed points (no redraw), bsde_solve only;
                      eta and q are not used.  The coefficients of such a
                      problem are its point values: p = n, coefficient row
                      k = y^{k-1} (row 0 zero); bsde_set_coefficients and
                      bsde_fit_values return BSDE_EUNSUPPORTED.  0: the
                      least-squares operator.                             */
} bsde_grid;

typedef enum {
    BSDE_FP64 = 0,       /* paths, driver, sums and update in FP64           */
    BSDE_FP32_PATHS = 1  /* paths, basis and driver in FP32; Monte Carlo
                            sums, least-squares update and coefficient
                            tables in FP64                                 */
} bsde_precision;

/* Creates a pricing problem and performs its one-time set-up: index set,
 * grid, basis matrix, rank-checked Householder QR, the pseudo-inverse
 * R^{-1} Q' and the derivative (channel) matrices, all uploaded to the
 * current HIP device.
 *   d         number of assets, 1 <= d <= 10 (a kernel must exist for
 *             (d, eta); BSDE_EUNSUPPORTED otherwise)
 *   sigma     volatility model (see bsde_sigma)
 *   r         interest rate
 *   payoff    payoff, strike, maturity and spots
 *   grid      points and basis (see bsde_grid)
 *   M         Monte Carlo paths per point and iteration, >= 1
 *   N         Euler steps per path, >= 1 (equal steps on [t_i, T])
 *   n_picard  Picard iterations K_it, >= 1
 *   penalty   omega of eq. bsde-penal-2 (0 = European option), >= 0
 *   seed      64-bit key of the Philox4x32-10 streams
 *   precision bsde_precision
 *   out       receives the handle (NULL on error)
 * Errors: BSDE_EINVAL, BSDE_ERANK, BSDE_ENOMEM, BSDE_EDEVICE,
 * BSDE_EUNSUPPORTED. */
bsde_status bsde_create_problem(int d, const bsde_sigma *sigma, double r,
                                const bsde_payoff *payoff,
                                const bsde_grid *grid, int M, int N,
                                int n_picard, double penalty,
                                unsigned long long seed, int precision,
                                bsde_problem *out);

/* Runs the remaining Picard iterations k_done..n_picard-1 (Algorithm
 * "algodetail": per-point Monte Carlo correction, eq. chat; least-squares
 * update, eq. alpha) on the given HIP stream (hipStream_t, NULL = the
 * default stream) and returns once they are complete.  Starting
 * coefficients are u^0 = 0 unless set with bsde_set_coefficients or
 * bsde_fit_values.  With redraw, each iteration first draws its points
 * and factorises their basis matrix on the device (waiting for the
 * previous iteration).  Errors: BSDE_EDEVICE, BSDE_ERANK (redrawn points
 * with a rank-deficient basis matrix). */
bsde_status bsde_solve(bsde_problem h, void *hip_stream);

/* Price u(t, log S) and dollar deltas Delta_j = e^{-x_j} d_{x_j} u (the
 * hedge of Section 5.1, in price units) from the last coefficients.
 *   nq     number of queries
 *   t      nq times
 *   S      nq * d prices, row-major (query-major)
 *   price  nq outputs; delta: nq * d outputs (row-major), may be NULL
 * Errors: BSDE_ESTATE if no iteration has run and no coefficients were
 * set, BSDE_EINVAL. */
bsde_status bsde_query_price_delta(bsde_problem h, int nq, const double *t,
                                   const double *S, double *price,
                                   double *delta);

/* Sizes of the problem: n points, p basis functions (full total-degree
 * set of the kernel; entries outside a hyperbolic set stay zero), C
 * derivative channels (u, d_t u, grad u, upper-triangular hessian). */
bsde_status bsde_problem_sizes(bsde_problem h, int *n, int *p, int *C);

/* The n * (d+1) grid points (t_i, x_i), row-major: with redraw, the
 * points of the last iteration run (iteration 0's before any solve). */
bsde_status bsde_get_points(bsde_problem h, double *pts);

/* Coefficients alpha^k (Chebyshev basis, p doubles) after k iterations,
 * 0 <= k <= k_done; k < 0 means the latest.  k_done receives the number
 * of completed iterations (may be NULL). */
bsde_status bsde_get_coefficients(bsde_problem h, int k, double *alpha,
                                  int *k_done);

/* Replaces the current coefficients and declares k_done iterations done
 * (checkpoint / resume; the random streams are keyed by k, so resuming
 * reproduces the remaining iterations). */
bsde_status bsde_set_coefficients(bsde_problem h, const double *alpha,
                                  int k_done);

/* Sets alpha = argmin ||y - B alpha|| for values y (n doubles) at the grid
 * points -- those bsde_get_points returns -- (least-squares fit of a known
 * function) and declares k_done iterations done. */
bsde_status bsde_fit_values(bsde_problem h, const double *y, int k_done);

/* Per-point correction c^k_i (eq. chat) and the sample variance of the
 * path terms a_m at iteration k (n doubles each; var may be NULL). */
bsde_status bsde_get_corrections(bsde_problem h, int k, double *c,
                                 double *var);

/* Path tiling of the Monte Carlo kernel: each point's M paths are split
 * over groups_per_point workgroups of 256 lanes, each lane running up to
 * paths_per_lane paths (0, 0 = automatic choice).  The result depends only
 * on the tiling through the summation order. */
bsde_status bsde_set_tiling(bsde_problem h, int groups_per_point,
                            int paths_per_lane);

/* Autotuner of the path tiling: times the path kernel of this problem (at
 * its current iteration, without changing its state) for every tiling of
 * 2^j paths per lane (j = 0..6) with enough groups to cover M (best of 4
 * timed launches each; a tiling with fewer groups replaces the current
 * choice only when more than 2% faster), keeps the choice for this problem
 * and records it for its kernel signature (d, eta,
 * precision, volatility kind, M, N, size class of n); problems created
 * afterwards with that signature start with it.  Outputs may be NULL:
 * groups and paths per lane chosen, and the path-kernel time in ms. */
bsde_status bsde_autotune(bsde_problem h, void *hip_stream, int *groups,
                          int *paths_per_lane, double *ms);

/* Tiling a problem will run with: groups per point and paths per lane as
 * set by bsde_set_tiling or bsde_autotune, or taken from a tiling recorded
 * for its signature when it was created (0, 0 = the automatic choice made at
 * each solve).  Errors: EINVAL for a null argument. */
bsde_status bsde_get_tiling(bsde_problem h, int *groups_per_point,
                            int *paths_per_lane);

/* Persistence of the tilings bsde_autotune has recorded in this process, so
 * that a later process starts its problems with them without timing again.
 * bsde_autotune_save writes every record to the text file path (replaced if
 * it exists), one line per signature: the architecture of the current
 * device (e.g. gfx950), d, eta, 10 q, precision, volatility kind, M, N, size
 * class of n, groups per point, paths per lane; lines starting with # are
 * comments.  bsde_autotune_load merges the records of path whose
 * architecture is that of the current device into this process's records
 * (a record of the same signature is replaced) and skips those of other
 * architectures; problems created afterwards start with them.  *count
 * (may be NULL) receives the number of records written or taken.  Errors:
 * EINVAL for a null path, a file that cannot be opened, or a malformed line
 * (load then changes nothing: every line is checked first, including that
 * the tiling covers M); EDEVICE when the device cannot be queried. */
bsde_status bsde_autotune_save(const char *path, int *count);
bsde_status bsde_autotune_load(const char *path, int *count);

/* Average duration in milliseconds of the last solve's kernels, measured
 * with HIP events on the solve's stream, per Picard iteration unless noted:
 * [0] Monte Carlo path kernel, [1] reduction of the per-point sums,
 * [2] projection R^{-1} Q' c, [3] coefficient/channel update, [4] whole
 * solve (not averaged).  What is measured depends on the timing level
 * (bsde_set_timing): level 1 (the default) times the path kernel, and
 * [1] then holds reduction, projection and update together ([2] = [3] =
 * 0); level 2 times each kernel; level 0 only the whole solve. */
bsde_status bsde_last_timings(bsde_problem h, double *ms5);

/* Timing level of later solves of h: 0 = whole solve only, 1 = also the
 * path kernel of every iteration (default), 2 = every kernel.  Each level
 * adds HIP event records to the stream between kernels, and each record
 * costs the stream a few microseconds.  Results do not depend on it.
 * Errors: EINVAL for a null handle or a level outside 0..2. */
bsde_status bsde_set_timing(bsde_problem h, int level);

/* Solves many problems together (hot-path row "batching"): all remaining
 * Picard iterations of every problem, with one persistent kernel launch per
 * iteration step and kernel signature (d, eta, precision, volatility kind)
 * that takes (problem, point, path-group) tiles from an atomic queue,
 * heaviest tiles first -- the GPU form of the dynamic per-point dispatch of
 * Section 4.3 -- and one launch each for the reductions and updates of all
 * problems.  Problems may differ in d, grid, M, N, iterations and
 * precision.  Each problem's result is identical to bsde_solve with the
 * same tiling.
 *   problems  count distinct handles (not owned)
 *   flags     BSDE_BATCH_GRAPH: capture the whole schedule as one hipGraph
 *             and replay it (on a library stream if hip_stream is NULL)
 *   ms        receives the GPU time of the batch in milliseconds (may be NULL)
 * Errors: BSDE_EINVAL, BSDE_EDEVICE. */
#define BSDE_BATCH_GRAPH 1
bsde_status bsde_solve_batch(bsde_problem *problems, int count,
                             void *hip_stream, int flags, double *ms);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * batched solve as bsde_solve_batch without graph capture and without
 * timing, whose descriptor tables and tile counters (the only device
 * memory bsde_solve_batch takes beyond the problems' own buffers) live in
 * a fixed workspace compiled into the library, 4 MiB per device, held on
 * each device used until the process ends, instead of memory from the
 * library's allocator.  The problems (created beforehand; their buffers
 * are the inputs and outputs) and their results are those of
 * bsde_solve_batch, bit for bit.  The tile counters are cleared by a fill
 * kernel at the start of every call.  Every call on a device uses that
 * device's one workspace: the library serialises calls of one process per
 * device (each returns after its kernels are done); work the caller
 * enqueues on other streams while a call runs must not depend on it.
 * Returns after completion.
 * Errors: BSDE_EINVAL (also when the batch's tables exceed the workspace:
 * about 2.4 KB per problem and iteration step), BSDE_ESTATE (a problem's
 * tiling was changed to one needing a larger per-group sum buffer than
 * it was created with), BSDE_EUNSUPPORTED (redrawn points, the kernel
 * operator), BSDE_EDEVICE. */
bsde_status bsde_solve_batch_noalloc(bsde_problem *problems, int count,
                                     void *hip_stream);

void bsde_destroy(bsde_problem h);

/* ------------------------------------------------------------------------
 * Request server (hot-path row "serving"): continuous batching of pricing
 * requests.  Requests are admitted while their device footprint fits the
 * HBM budget and fewer than max_inflight are in flight; set-up threads
 * build admitted problems while the GPU works; one engine thread advances
 * all in-flight problems with the batched kernels (bsde_solve_batch) step
 * by step, so requests arriving while others run join at the next step.
 * A step lasts about one Picard iteration of its most expensive problem;
 * cheaper problems run several of their iterations in it (at most 16).  Each problem's coefficients stay resident on the
 * device across its iterations.  A request's result is identical whether it
 * runs alone or in a mix.  All server calls are thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct bsde_server_s *bsde_server; /* owned by the library */

/* One request: the arguments of bsde_create_problem plus a query point. */
typedef struct {
    int d;
    bsde_sigma sigma;
    double r;
    bsde_payoff payoff;
    bsde_grid grid;
    int M, N, n_picard;
    double penalty;
    unsigned long long seed;
    int precision;
    double query_t;          /* time of the price/delta query              */
    const double *query_S;   /* d prices, or NULL for the spots S0          */
} bsde_request;

typedef struct {
    int status;              /* bsde_status of the request                  */
    double price;            /* u(query_t, log query_S)                     */
    double delta[10];        /* dollar deltas (first d entries)             */
    double latency_ms;       /* submit to completion                        */
    double queue_ms;         /* submit to admission                         */
    int engine_steps;        /* engine steps the request took part in       */
} bsde_result;

typedef struct {
    double p50_ms, p99_ms;     /* request latency percentiles              */
    double requests_per_s;     /* completed / (first submit .. last done)  */
    double path_steps_per_s;   /* sum of n M N K_it over the same span      */
    long completed, engine_steps, in_flight, pending;
    size_t reserved_bytes;     /* device bytes reserved by admitted requests */
} bsde_server_stats_t;

/* hbm_budget_bytes: device bytes the server may reserve for admitted
 * problems; max_inflight: problems in set-up or on the GPU at once;
 * setup_threads: host threads building problems (0 = 4).  Uses the HIP
 * device current at the call.  Errors: BSDE_EINVAL, BSDE_EDEVICE. */
bsde_status bsde_server_create(size_t hbm_budget_bytes, int max_inflight,
                               int setup_threads, bsde_server *out);
/* Queues a request (arrays are copied); ticket receives its id.  Errors:
 * BSDE_EINVAL, BSDE_EUNSUPPORTED (a grid with redraw: such problems need
 * a host-side factorisation between iterations and run through bsde_solve
 * only); errors of the problem itself arrive through bsde_server_poll. */
bsde_status bsde_server_submit(bsde_server s, const bsde_request *req,
                               unsigned long long *ticket);
/* Result of a ticket; with wait = 0 returns BSDE_EBUSY while it runs.  A
 * ticket can be collected once. */
bsde_status bsde_server_poll(bsde_server s, unsigned long long ticket,
                             int wait, bsde_result *out);
bsde_status bsde_server_stats(bsde_server s, bsde_server_stats_t *out);
/* Stops admitting, finishes the problems already built, frees everything;
 * requests not yet admitted are dropped. */
void bsde_server_destroy(bsde_server s);
const char *bsde_status_string(bsde_status s);
/* Human-readable detail of the last error on this thread. */
const char *bsde_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
