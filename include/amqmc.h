/*
 * amqmc.h — C-ABI of the MI355X quasi-Monte Carlo American option engine.
 *
 * Method: Cvetanoska & Stojanovski, "Using High Performance Computing and
 * Monte Carlo Simulation for Pricing American Options".  One call values one
 * option on n_paths quasi-random GBM paths observed at n_dates exercise dates:
 *   - quasi-random points mapped to N(0,1) by Moro's inverse cumulative normal
 *     (Section III.D);
 *   - GBM on the Bermudan grid t_k = kT/M, k = 1..M (Sections III.E and V,
 *     eq. (9), taken as the exact lognormal map built by a Brownian bridge);
 *   - backward induction over the dates (Section V, eqs. (10)-(11)) with the
 *     continuation value estimated by least squares over in-the-money paths
 *     (the regression approach the paper cites as [9], [12], [19]);
 *   - the discounted mean of eqs. (6)-(8).
 *
 * Quasi-random points: unscrambled Sobol (Joe–Kuo direction numbers), Gray
 * code order, path i uses sequence index i+1; dimension 1 drives W(T) and
 * dimension q+1 the q-th breadth-first bisection node of the bridge.
 *
 * All entry points return AM_OK (0) or a negative error code; on error no
 * output is written and am_last_error() describes the failure.  Host
 * pointers are owned by the caller and only read or written during the call.
 */
#ifndef AMQMC_H
#define AMQMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Option and model parameters (Section III.C notation in brackets). */
typedef struct am_params {
    double S0;              /* spot at t0 [S_0], > 0 */
    double K;               /* strike [X], > 0 */
    double r;               /* continuously compounded rate [r], finite */
    double sigma;           /* volatility [v], > 0 */
    double T;               /* expiry [T], > 0 */
    int32_t is_call;        /* 1 call, 0 put */
    int32_t allow_exercise; /* 1: exercise at t_1..t_{M-1} (least squares) and at
                               t0 (price = max(h(S0), mean)); 0: European */
} am_params;

/* Regression basis: functions of x = S/K.  MONOMIAL: 1, x, .., x^d.
 * LAGUERRE: exp(-x/2) L_n(x), n = 0..d (weighted Laguerre functions).
 * p = degree + 1 functions, 0 <= degree <= AM_MAX_DEGREE.  The engine solves
 * in an equivalent basis of the same span (standardised x); fitted values,
 * and hence prices, do not depend on that choice. */
typedef struct am_basis {
    int32_t kind;
    int32_t degree;
} am_basis;

enum { AM_BASIS_MONOMIAL = 0, AM_BASIS_LAGUERRE = 1 };
enum { AM_MAX_DEGREE = 6 };

/* Arithmetic of the bulk path data.
 *   AM_FP64:      everything binary64.
 *   AM_FP32_BULK: path values and per-path cashflows (discounted to t0)
 *                 stored in binary32, each rounded once from its binary64
 *                 value (half the HBM traffic and footprint); the inverse
 *                 normal, the bridge, the exponent and every step of the
 *                 backward induction in binary64 (the least-squares fit and
 *                 the exercise test react to relative perturbations near
 *                 1e-8, and to single-ulp changes of the stored values, for
 *                 some options).  The result is the method on binary32
 *                 storage; for a few ill-conditioned options that storage
 *                 alone moves the price by more than 2e-3 from the binary64
 *                 result. */
enum { AM_FP64 = 0, AM_FP32_BULK = 1 };

/* Storage rule for small requests.  With fewer than AM_FP32_MIN_PATHS paths a
 * single exercise decision that rounds the other way in binary32 storage
 * moves the price by up to (largest payoff)/N, which alone can exceed the
 * FP32-bulk tolerance of 2e-3 absolute.  AM_FP32_BULK requests below that
 * path count are therefore stored in binary64 (they are latency-bound, so the
 * doubled bytes cost nothing measurable); every pricing entry point applies
 * the rule (single option, randomised QMC per replicate, each option of a
 * batch, each served request), workspace sizes and layouts included.  The
 * paper's estimator (no regression, no decision feedback) stores as asked. */
enum { AM_FP32_MIN_PATHS = 16384 };

/* The storage type (AM_FP64 or AM_FP32_BULK) a pricing request of n_paths
 * paths gets under that rule; -1 for an unknown dtype. */
int32_t am_storage_dtype(int64_t n_paths, int32_t dtype);

enum {
    AM_OK = 0,
    AM_EINVAL = -1,      /* a parameter is out of range or not finite */
    AM_ENOMEM = -2,      /* device or host allocation failed */
    AM_EDEVICE = -3,     /* a HIP call failed */
    AM_EDIM = -4,        /* n_dates or n_paths beyond what the engine supports */
    AM_EWORKSPACE = -5,  /* workspace too small or misaligned */
    AM_ETIMEOUT = -6     /* a device-side wait exceeded its bound */
};

/* Price one option, synchronously, on the current HIP device.  Uses a
 * library-owned stream and workspace (grown on demand, kept per device).
 * Writes *price and *std_err (naive iid standard error sd(PV)/sqrt(N); 0
 * when exercise at t0 wins).  Thread-safe; calls on one device serialise. */
int am_price_american(const am_params *params, int64_t n_paths, int32_t n_dates,
                      am_basis basis, int32_t dtype, double *price, double *std_err);

/* Workspace bytes am_price_american_ex needs for this shape. */
size_t am_workspace_bytes(int64_t n_paths, int32_t n_dates, am_basis basis, int32_t dtype);

/* Offsets (bytes from the workspace base) of the regions a test or tool may
 * read after a call, in this order:
 *   [0] S: paths, [n_dates][ld] of double or float, as am_storage_dtype()
 *       names for (n_paths, dtype),
 *       row k-1 holds t_k, column i holds path i;
 *   [1] PV: [ld] per-path cashflow discounted to t0, same type as S;
 *   [2] per-date records: [n_dates+1][40] double; row k (1 <= k < n_dates)
 *       holds the date's regression: [0..7] coefficients of the fitted value
 *       (cashflow discounted to t0) in the engine's standardised basis, [8] 1
 *       if solved / 0 if the date allowed no exercise, [9] in-the-money count,
 *       [10..30] the moment sums it was solved from, [32..36] group 0's
 *       device clock stamps (100 MHz) of the date's phases: moments summed
 *       in the group, device-wide totals in hand, solved, the next date's
 *       Gram part summed (tiles that overlap it with the sum; else equal to
 *       [32]), the date's pass started;
 *   [3] result: [8] double {price, std_err, mean_pv, t0_exercise, n_skipped,
 *       error_flag, 0, 0};
 *   [4] ld (elements, not bytes); [5] total bytes.
 * Returns AM_OK or AM_EINVAL. */
int am_workspace_layout(int64_t n_paths, int32_t n_dates, am_basis basis, int32_t dtype,
                        size_t out[6]);

/* Price one option asynchronously on `hip_stream` (a hipStream_t; NULL is the
 * null stream) using the caller's device workspace d_workspace of ws_bytes
 * (>= am_workspace_bytes, 256-byte aligned, on the current device).  The
 * workspace must not be shared by calls that may overlap.  Calls enqueued
 * on different streams of one device may overlap in generation; their
 * sweeps (each holding every CU) run one after another, in enqueue order.
 * A sweep kept from being fully resident by other work on the device waits
 * boundedly and then fails with AM_ETIMEOUT.  If h_out is
 * non-NULL the call waits for the stream and writes h_out[0] = price,
 * h_out[1] = std_err; if NULL it returns after enqueueing and the result
 * stays in the workspace result region. */
int am_price_american_ex(const am_params *params, int64_t n_paths, int32_t n_dates,
                         am_basis basis, int32_t dtype, void *d_workspace, size_t ws_bytes,
                         void *hip_stream, double *h_out);

/* Size of the fixed device workspace of am_price_american_noalloc: 128 MiB
 * on each device the library runs on, held until the process ends. */
enum { AM_SCRATCH_BYTES = 134217728 };

/* Set up the current device for the library: direction-number table,
 * stream, the event that orders single-option sweeps, the device address of
 * the allocation-free entry point's workspace, and every single-option
 * kernel's code loaded on the device.  Allocates; idempotent; any thread.
 * Needed once per device (and again after am_shutdown) before
 * am_price_american_noalloc; the other entry points set up lazily. */
int am_init(void);

/* For callers that cannot allocate device memory (work under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): prices
 * exactly as am_price_american_ex (same kernels, same tiles: bitwise the
 * same price and std_err) but its workspace is a fixed array of
 * AM_SCRATCH_BYTES that the library holds on the device, and the call
 * allocates nothing: no hipMalloc, hipFree, hipHostMalloc, event or stream
 * creation.  am_init must have run on the current device (AM_EINVAL
 * otherwise).  The bridge schedule for n_dates is copied into the array
 * from host memory on hip_stream (a hipStream_t; NULL is the null stream);
 * the call waits for hip_stream and writes h_out[0] = price, h_out[1] =
 * std_err (h_out must be non-NULL).  A shape whose am_workspace_bytes plus
 * 64 * n_dates exceeds AM_SCRATCH_BYTES fails with AM_EWORKSPACE (for
 * binary64 storage about 2^17 paths x 125 dates, binary32 2^18 x 125).
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (the kernels clear what has to start at zero); calls that
 * overlap on one device, from two threads or on two streams, race on it and
 * must be serialised by the caller.  am_profile_* does not time this entry
 * point. */
int am_price_american_noalloc(const am_params *params, int64_t n_paths, int32_t n_dates,
                              am_basis basis, int32_t dtype, void *hip_stream, double *h_out);

/* Randomised quasi-Monte Carlo (reading of Section III.D, where the
 * quasi-random arrays are permuted by a linear congruential generator to make
 * the per-path samples statistically independent): n_rep independent
 * pricings, replicate r using the points x XOR h_shifts[r*n_dates + j] in
 * dimension j (a random digital shift; the caller draws the shifts, e.g.
 * uniform 32-bit words) mapped to cell midpoints u = (x + 1/2) 2^-32.
 * h_out (n_rep + 2 doubles, or NULL for asynchronous use) receives the mean
 * of the replicate prices, sd/sqrt(n_rep) across replicates (an honest
 * error bar), then the replicate prices.  1 <= n_rep <= 64.  The replicates
 * run one after another in the single-option layout; workspace as in
 * am_price_american_ex. */
int am_price_american_rqmc(const am_params *params, int64_t n_paths, int32_t n_dates,
                           am_basis basis, int32_t dtype, int32_t n_rep, const uint32_t *h_shifts,
                           void *d_workspace, size_t ws_bytes, void *hip_stream, double *h_out);

/* The same replicates all at once: a batch of identical options, each with
 * its own digital shift (one generation launch and one persistent sweep, as
 * am_price_batch), the mean and error bar formed on the host in the order
 * and arithmetic of am_price_american_rqmc's final step.  Replicate prices
 * agree with am_price_american_rqmc's to rounding (the tiles sum in a
 * different order).  The batch tile is the larger one while the replicates
 * give at least one tile per compute unit at that size, else the smaller.
 * Workspace: am_rqmc_workspace_bytes, 256-byte aligned; h_out (n_rep + 2
 * doubles) is required; returns once the results are in. */
int am_price_rqmc_batch(const am_params *params, int64_t n_paths, int32_t n_dates, am_basis basis,
                        int32_t dtype, int32_t n_rep, const uint32_t *h_shifts, void *d_workspace,
                        size_t ws_bytes, void *hip_stream, double *h_out);

/* Workspace bytes of am_price_rqmc_batch (0 if the arguments are invalid). */
size_t am_rqmc_workspace_bytes(int64_t n_paths, int32_t n_dates, am_basis basis, int32_t dtype,
                               int32_t n_rep);

/* The paper's own estimator (Section V, eqs. (10)-(11)) on the same
 * quasi-random paths: n_points exercise points t_i = i T/(n_points+1); at the
 * last point the value is max(h(S), Black–Scholes value over the remaining
 * interval), earlier c_i = max(h(S_i), exp(-r dt) c_{i+1}); price =
 * exp(-r dt) * mean(c_1) and its naive standard error.  Perfect foresight
 * along each path, so an upper-bias estimate (the paper calls it an upper
 * bound).  Uses the workspace of am_workspace_bytes(n_paths, n_points, any
 * basis, dtype); params->allow_exercise is ignored.  Stream, workspace and
 * h_out semantics as in am_price_american_ex. */
int am_price_paper_estimator(const am_params *params, int64_t n_paths, int32_t n_points,
                             int32_t dtype, void *d_workspace, size_t ws_bytes, void *hip_stream,
                             double *h_out);

/* ---------------------------------------------------------------------- */
/* Batches: many options in one generation launch and one persistent sweep. */
/* ---------------------------------------------------------------------- */

/* One option of a batch. */
typedef struct am_option {
    am_params params;
    int64_t n_paths;
    int32_t n_dates;
    int32_t reserved;       /* 0 */
} am_option;

/* Workspace bytes for am_price_batch on these options (0 if invalid). */
size_t am_batch_workspace_bytes(const am_option *opts, int32_t n_opts, am_basis basis,
                                int32_t dtype);

/* Price n_opts options, each exactly as am_price_american_ex defines it
 * (same points, same estimator), sharing one basis and dtype.  Paths of all
 * options are generated in one launch; the backward sweeps run in one
 * persistent launch in which workgroups claim (option, tile) slots and each
 * option synchronises only its own tiles, so options of uneven path and date
 * counts overlap on the device.  Each option's result depends only on its own
 * data (fixed-order reductions): the same alone and in any mix.  Under
 * AM_FP32_BULK, options below AM_FP32_MIN_PATHS paths form a second
 * sub-batch stored in binary64 (a second generation and sweep launch on the
 * stream; am_batch_workspace_bytes covers both).  h_out (2 * n_opts
 * doubles, or NULL to return after enqueueing) receives price and std_err
 * per option in the caller's order.  Fails with AM_EDIM if one option needs
 * more tiles than the device holds resident. */
int am_price_batch(const am_option *opts, int32_t n_opts, am_basis basis, int32_t dtype,
                   void *d_workspace, size_t ws_bytes, void *hip_stream, double *h_out);

/* Thread-local description of the last failure on this thread; valid until
 * the next call on the same thread.  Never NULL. */
const char *am_last_error(void);

/* Largest n_dates the engine supports (bounded by the Sobol table and the
 * on-chip generation tables). */
int am_max_dates(void);

/* Largest n_paths one call supports at this precision on the current device
 * (paths are kept resident on chip during the backward sweep). */
int64_t am_max_paths(int32_t dtype);

/* ---------------------------------------------------------------------- */
/* Inspection entry points used by the parity tests.                       */
/* ---------------------------------------------------------------------- */

/* Run the generation kernel in a diagnostic mode on the current device and
 * copy its raw output to host_out ([count_dims][n_paths], row-major):
 *   what = 1: Sobol integers x_j(i+1) for dims j = 1..n_dims;
 *   what = 2: inverse-normal values z as double (from the given dtype);
 *   what = 0: the paths S as double (row k-1 = t_k), for params.
 * host_out must hold n_dims * n_paths elements (uint32 for what = 1, double
 * otherwise).  Synchronous. */
int am_debug_generate(int32_t what, const am_params *params, int64_t n_paths, int32_t n_dims,
                      int32_t dtype, void *host_out);

/* Host-side bridge schedule for n_dates (no device work): node q in
 * construction order gets date m[q], Sobol dimension dim[q] (0-based), and
 * weights so that W(t_m) = wl*W(t_left) + wr*W(t_right) + sd*sqrt(T/M)*z.
 * Arrays hold n_dates entries. */
int am_debug_schedule(int32_t n_dates, int32_t *m, int32_t *dim, int32_t *left,
                      int32_t *right, double *wl, double *wr, double *sd);

/* Kernel timing for measurement tools.  While enabled on the calling thread,
 * each pricing call records HIP events on its stream before the generation
 * kernel, between the two kernels and after the sweep kernel.
 * am_profile_read waits for the recorded events and returns the summed
 * milliseconds of generation (ms[0]) and sweep (ms[1]) and the number of
 * calls timed since the last read, then clears the record.  Enabling or
 * disabling also clears it. */
int am_profile_enable(int32_t on);
int am_profile_read(double ms[2], int64_t *calls);

/* Time the batch with each candidate tile shape (paths per thread: FP32 16
 * and 64, FP64 8 and 32; two timed runs each after a warm-up), remember the
 * faster one for this shape class (precision, degree, batch size and total
 * path-steps rounded to powers of two) for later am_price_batch calls in the
 * process, and return it in *best_ppt (ms_out: mean milliseconds per
 * candidate, may be NULL).  Synchronous on hip_stream. */
int am_batch_autotune(const am_option *opts, int32_t n_opts, am_basis basis, int32_t dtype,
                      void *d_workspace, size_t ws_bytes, void *hip_stream, int32_t *best_ppt,
                      double ms_out[2]);

/* A batch captured once as a HIP graph (table uploads from pinned staging,
 * both kernels, result download) and replayed with one launch.  The
 * options, workspace and tile choice are fixed at capture. */
typedef struct am_batch_graph am_batch_graph;
int am_batch_graph_create(const am_option *opts, int32_t n_opts, am_basis basis, int32_t dtype,
                          void *d_workspace, size_t ws_bytes, am_batch_graph **out);
int am_batch_graph_launch(am_batch_graph *graph, void *hip_stream);
/* Wait for the last launch and write price, std_err per option (2*n doubles). */
int am_batch_graph_results(am_batch_graph *graph, double *h_out);
int am_batch_graph_destroy(am_batch_graph *graph);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of pricing requests under an HBM budget.    */
/* ---------------------------------------------------------------------- */
typedef struct am_server am_server;

typedef struct am_server_config {
    size_t hbm_budget_bytes;       /* device pool allocated once; workspaces are carved from it */
    double max_batch_path_steps;   /* cap on sum n_paths*n_dates per launched batch */
    int32_t max_batch_requests;    /* cap on requests per launched batch */
    int32_t n_streams;             /* batches in flight at once (1..8) */
    am_basis basis;                /* shared by every request */
    int32_t dtype;
    int32_t large_tile;            /* 0: the smaller batch tile; 1: the larger (see am_server_create) */
} am_server_config;

typedef struct am_result {
    uint64_t request_id;
    double price, std_err;
    double t_arrival;              /* server clock (am_server_now), seconds */
    double t_launch;               /* when its batch was enqueued */
    double t_done;                 /* when completion was observed */
    int32_t status;                /* AM_OK, AM_ENOMEM (larger than the budget), ... */
    int32_t reserved;
} am_result;

/* Start a server on the current device: allocates the pool and starts a
 * dispatcher thread.  Requests wait in arrival order; whenever a stream is
 * free, the longest prefix of waiting requests whose batch workspace fits in
 * the free pool (and under the batch caps) is launched as one batch
 * (am_price_batch's kernels, persistent grid limited to 1/n_streams of the
 * device so in-flight batches run side by side); completed batches return
 * their memory.  A request whose sweep needs more workgroups than that share
 * runs alone on the whole device once every stream is idle (later requests
 * wait behind it).  Paths and cashflows stay resident in the pool until a
 * request completes.  Results are those of am_price_batch, hence identical
 * to pricing the request alone with the same batch tile.  The tile is fixed
 * per server, whatever am_batch_autotune chose: the smaller (FP32 bulk 16
 * paths per thread, FP64 8), whose sweeps spread a request of few paths over
 * four times the workgroups of the larger, or with large_tile the larger
 * (64 and 32; am_price_batch's default), which admits requests of four times
 * the paths (am_server_submit).  Fails with AM_EINVAL for large_tile other
 * than 0 or 1. */
int am_server_create(const am_server_config *cfg, am_server **out);

/* Queue one request (non-blocking, thread-safe).  t_arrival < 0 means now.
 * Returns AM_EDIM (and queues nothing) for a request whose sweep would not
 * be resident even on the whole device; a request larger than the HBM
 * budget is queued and completes with status AM_ENOMEM. */
int am_server_submit(am_server *server, const am_option *opt, uint64_t request_id, double t_arrival);

/* Move up to max_out completed results into out; *n_out receives the count. */
int am_server_poll(am_server *server, am_result *out, int32_t max_out, int32_t *n_out);

/* Server clock in seconds (monotonic). */
double am_server_now(void);

/* out: {batches launched, requests launched, path-steps launched, pool bytes in use}. */
int am_server_stats(am_server *server, double out[4]);

/* Finish every queued request, stop the dispatcher, free the pool.  Results
 * not yet polled are discarded.  Returns the first fatal error, if any. */
int am_server_destroy(am_server *server);

/* Release what the library holds for the life of the process: per device
 * the direction-number table, the bridge schedules, the synchronous entry
 * point's workspace and stream and the event that orders single-option
 * sweeps; the pinned result buffers and profiling events of every thread.
 * Waits for the library's own streams first.  Call it with no other library
 * call in flight and no server alive (AM_EINVAL otherwise); a later call
 * sets the state up again.  The Python binding calls it at interpreter exit,
 * so nothing of the library is left for the HIP runtime (and a profiler
 * attached to it) to tear down after its own finalisation. */
int am_shutdown(void);

/* Tuning hook: paths per thread of the batch sweep on this thread (FP32: 16
 * or 64, FP64: 8 or 32) for am_price_batch and am_price_rqmc_batch; 0
 * restores their defaults (see each).  Servers keep the tile they were
 * created with.  Results of one option are identical for a given choice;
 * different choices change the reduction order (differences at rounding
 * level). */
void am_debug_set_batch_ppt(int32_t ppt);

/* Tuning hook: allow (1, the default) or forbid (0) 512-thread workgroups in
 * single-option sweeps on this thread.  The tile size chosen for a given
 * n_paths may differ, which changes the reduction order (differences at
 * rounding level). */
void am_debug_set_sweep_wide(int32_t allow);

/* Test hook: single-option sweeps on this thread use the tile of wg threads
 * per group and ppt paths per thread (one of the built tiles, e.g. binary32
 * 512 x 64 or 512 x 128, the slab-resident monomial forms), or fail with
 * AM_EDIM where it does not apply (row padding, residency); wg = 0 restores
 * the cost model's choice.  The tile changes the reduction order
 * (differences at rounding level). */
void am_debug_set_sweep_tile(int32_t wg, int32_t ppt);

/* Test hook: bound the device-side barrier waits of subsequent calls on this
 * thread to `spins` polls (0 restores the default).  A wait that runs out
 * makes the call return AM_ETIMEOUT after every workgroup has exited. */
void am_debug_set_spin_limit(uint32_t spins);

#ifdef __cplusplus
}
#endif
#endif
