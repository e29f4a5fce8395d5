/*
 * krr.h -- C ABI of a batched, partitioned kernel ridge regression library
 * for AMD Instinct MI355X (gfx950).
 *
 * Method: You, Demmel, Hsieh, Vuduc, "Accurate, Fast and Scalable Kernel
 * Ridge Regression on Parallel and Distributed Systems" (ICS'18).  The
 * training set is split into p partitions (K-means: Section 2.4, Algorithm 2;
 * K-balance: Section 4.3, Algorithm 4); every partition gets its own kernel
 * ridge regression model (Section 2.3, Eq. 6, Algorithm 1); a test point is
 * predicted by the model of its nearest partition centre (KKRR2, Section 4.2;
 * BKRR2, Algorithm 5) or by the average of all models (KKRR, Section 4.1);
 * the best (sigma, lambda) is the one with the lowest MSE (Eq. 3,
 * Algorithm 5).  On one GPU the p partition models of every (sigma, lambda)
 * setting are solved as one ragged batch.
 *
 * Conventions shared by every call:
 *   - Every call returns krr_status: 0 on success, a negative code on error.
 *     No C++ exception crosses this interface.  krr_last_error() returns a
 *     human-readable message for the last failing call on a context.
 *   - Array arguments marked "device" are device pointers on the context's
 *     GPU, owned by the caller, row-major, and must stay valid until the work
 *     queued on `stream` has finished.  Arguments marked "host" are host
 *     pointers.  Outputs are allocated by the caller with the stated sizes.
 *   - Work is queued on `stream` (NULL = the default stream).  Calls that
 *     return host outputs synchronise `stream` before returning; the others
 *     are asynchronous unless stated.
 *   - Argument errors (sizes < 1, p outside [1, n], sigma <= 0, a lambda that
 *     is not finite, null pointers, unknown enum values) return KRR_EINVAL
 *     before any work is queued.
 *   - One host thread may use a context at a time.  Calls from several
 *     threads on different contexts are independent.
 */
#ifndef KRR_H_
#define KRR_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct krr_ctx_s*   krr_ctx;    /* device, workspace pool, options, last error */
typedef struct krr_model_s* krr_model;  /* one fitted (sigma, lambda) over all partitions */

typedef enum {
  KRR_OK = 0,
  KRR_EINVAL = -1,    /* bad argument */
  KRR_ENOMEM = -2,    /* device allocation failed */
  KRR_EBUDGET = -3,   /* the call would exceed the context's HBM budget */
  KRR_ENOTSPD = -4,   /* K + lambda I not positive definite in the working precision */
  KRR_ENOCONV = -5,   /* iterative refinement did not reach refine_tol */
  KRR_EDEVICE = -6,   /* a HIP runtime call failed */
  KRR_ESTATE = -7     /* object used in a state that does not allow the call */
} krr_status;

typedef enum { KRR_F32 = 0, KRR_F64 = 1 } krr_dtype;

/* Partitioning methods.  KMEANS: k-means++ seeding + Lloyd (Algorithm 2);
 * KBALANCE: K-means followed by the capacity-ceil(n/p) greedy pass and the
 * centre recompute (Algorithm 4); GIVEN: assign to caller-supplied centres
 * (the assignment step of Algorithm 2); RANDOM: DC-KRR's divide step
 * (Algorithm 3): the rows are shuffled by a permutation keyed by `seed`
 * (Feistel network with SplitMix64 round keys, cycle-walked to [0, n)) and
 * partition j takes the shuffled rows [floor(j n/p), floor((j+1) n/p));
 * centroids are the member means (lloyd_iters is ignored).  Algorithm 3
 * then averages all models: KRR_ROUTE_AVERAGE with lambda_times_m = 1.
 * KBALANCE_APPROX: the approximate parallel K-balance of Section 4.3: the
 * same K-means centres; the samples in input order are split into p even
 * segments, rows [floor(q n/p), floor((q+1) n/p)) (one per node), each
 * segment runs the greedy pass on its own with capacity ceil(n_q/p) per
 * centre (the paper's n/p^2), then the centres are recomputed as member
 * means.  A partition holds at most p * ceil(ceil(n/p)/p) points, and
 * exactly n/p when p^2 divides n. */
typedef enum {
  KRR_PART_KMEANS = 0,
  KRR_PART_KBALANCE = 1,
  KRR_PART_GIVEN = 2,
  KRR_PART_RANDOM = 3,
  KRR_PART_KBALANCE_APPROX = 4
} krr_part;

/* Working precision of a fit.
 * FP64:  kernel matrix, Cholesky and solves in FP64.
 * FP32:  kernel matrix stored and factored in FP32 (FP32 matrix cores),
 *        diagonal blocks factored in FP64; no refinement.
 * MIXED: FP32 storage, BF16 matrix-core trailing updates with FP32
 *        accumulation, FP64 diagonal blocks, then iterative refinement with an
 *        FP64 residual r = y - (K + lambda I) alpha until alpha's estimated
 *        error is within refine_tol (see krr_fit_params).  A system whose
 *        BF16-updated factor is not positive definite, whose kappa_est exceeds
 *        128 (BF16 rounding would not contract), or whose refinement stops
 *        halving the residual is refactored with FP32 updates and refined again
 *        (krr_part_info.fallback = 1). */
typedef enum { KRR_PREC_FP64 = 0, KRR_PREC_FP32 = 1, KRR_PREC_MIXED = 2 } krr_prec;

/* Prediction routes.  NEAREST: model of the nearest centre (KKRR2 / BKRR2,
 * Section 4.2, Algorithm 5).  AVERAGE: mean of all p models (KKRR / DC-KRR,
 * Section 4.1, Algorithm 3).  ALL: the k x p matrix of every model's
 * prediction.  LABEL (krr_select only: it needs the labels): per point, the
 * one of the p models whose prediction is closest to the point's label
 * (BKRR3 / KKRR3, Section 4.4, Algorithm 6; the error lower bound of the
 * partitioned methods). */
typedef enum { KRR_ROUTE_NEAREST = 0, KRR_ROUTE_AVERAGE = 1, KRR_ROUTE_ALL = 2, KRR_ROUTE_LABEL = 3 } krr_route;

/* Table 1: Gaussian exp(-||a-b||^2 / (2 sigma^2)); linear a^T b; polynomial
 * (kernel_a a^T b + kernel_r)^kernel_degree; sigmoid tanh(kernel_a a^T b +
 * kernel_r).  The sigmoid kernel is not positive semi-definite in general: a
 * system whose K + lambda I is not positive definite is reported as
 * KRR_ENOTSPD with its failing pivot, like any other, unless its setting
 * asks for the LU solve (krr_fit_params.indefinite). */
typedef enum { KRR_KERNEL_GAUSSIAN = 0, KRR_KERNEL_LINEAR = 1, KRR_KERNEL_POLYNOMIAL = 2,
               KRR_KERNEL_SIGMOID = 3 } krr_kernel;

typedef struct {
  double  sigma;          /* Gaussian width (> 0; ignored by the linear kernel) */
  double  lambda;         /* diagonal shift (finite; see lambda_times_m).  A negative
                             shift can make the system indefinite, which is reported
                             as KRR_ENOTSPD with the failing pivot */
  int32_t kernel;         /* krr_kernel */
  int32_t prec;           /* krr_prec */
  double  refine_tol;     /* MIXED: target relative residual and relative error of alpha
                             (e.g. 1e-6).  A system converges when ||r||/||y|| <= refine_tol
                             and either kappa_bound * ||r||/||y|| <= refine_tol or, once
                             corrections have been applied, the error estimate from their
                             sizes (||delta|| rho / (1 - rho) / ||alpha||, rho the ratio of the
                             last two corrections) is <= refine_tol */
  int32_t max_refine;     /* MIXED: at most this many refinement steps (0 = none) */
  int32_t lambda_times_m; /* 1: shift is lambda * m_j per partition (Algorithms 3, 5, 6);
                             0: shift is lambda (Eq. 6 with the 1/n folded in) */
  double  kernel_a;       /* POLYNOMIAL, SIGMOID: scale a of the inner product (finite) */
  double  kernel_r;       /* POLYNOMIAL, SIGMOID: offset r (finite) */
  int32_t kernel_degree;  /* POLYNOMIAL: integer degree d in [1, 64] */
  int32_t indefinite;     /* 0 or 1.  1: a system whose Cholesky factorisation meets a
                             non-positive pivot (an indefinite K + lambda I, e.g. from the
                             sigmoid kernel) is solved instead by Gaussian elimination (the
                             paper's other solver, Implementation Details): LU with partial
                             pivoting of the FP64 system, with no refinement; it reports
                             solver = 1 and status KRR_OK, or KRR_ENOTSPD if a pivot column
                             is entirely zero.  0: such a system is reported as KRR_ENOTSPD */
} krr_fit_params;

typedef struct {
  int32_t partition;      /* partition index j */
  int32_t param;          /* index into the params array */
  int32_t m;              /* partition size */
  int32_t status;         /* KRR_OK, KRR_ENOTSPD or KRR_ENOCONV */
  int32_t failed_pivot;   /* 1-based column of the first non-positive pivot, 0 if none */
  int32_t refine_iters;   /* refinement steps taken (MIXED) */
  int32_t fallback;       /* MIXED: 0 = BF16 trailing updates sufficed; 1 = the system was
                             refactored with FP32 trailing updates after its BF16 factor
                             was not positive definite or refinement stalled */
  int32_t solver;         /* 0: Cholesky (Eq. 6); 1: LU with partial pivoting (an indefinite
                             system of a setting with indefinite = 1; failed_pivot then keeps
                             the Cholesky pivot that rejected it, and rel_residual, err_est
                             and kappa_bound are -1) */
  double  rel_residual;   /* ||y - (K + lambda I) alpha|| / ||y|| in FP64 (MIXED; -1 otherwise) */
  double  kappa_est;      /* (max_i L_ii / min_i L_ii)^2 of the factor: a lower bound of the
                             2-norm condition number of K + lambda I (1 for an empty system) */
  double  err_est;        /* MIXED: estimated relative error of alpha when refinement stopped
                             (the smaller of kappa_bound * ||r||/||y|| and the estimate from
                             the corrections, see refine_tol); -1 otherwise */
  double  kappa_bound;    /* MIXED: an upper bound of the 2-norm condition number of the FP64
                             system (Gershgorin's discs; for a positive semi-definite kernel the
                             smallest eigenvalue is also at least lambda); inf when no bound is
                             available; -1 otherwise */
} krr_part_info;

/* Tunables (krr_set_option).  Values apply to later calls on the context. */
typedef enum {
  KRR_OPT_PANEL_TILES = 0,  /* Cholesky panel width in 64-wide tiles (1..64; 0, the default:
                               24 in mixed precision, 16 in FP32 and FP64) */
  KRR_OPT_SERIAL_FIT = 1,   /* 1: factor the systems one after another, one launch
                               sequence per (partition, setting) -- the plain per-partition
                               baseline; 0 (default): one batched launch sequence */
  KRR_OPT_SYNC_CHECK = 2,   /* 1: synchronise after every launch and report faults (debug) */
  KRR_OPT_TIMING = 3,       /* HIP-event timing of kernel launches: 0 off, 1 the matrix-core
                               factorisation updates only, 2 every timed kernel class;
                               setting it clears the record (see krr_timing_report) */
  KRR_OPT_PERSISTENT = 4,   /* 1: the batched factorisation runs as one persistent launch:
                               every stage of every system from device task queues, each
                               system advancing on its own (ragged batches need no barrier
                               between systems); 0 (default): one launch per stage for the
                               whole batch.  Both give identical results */
  KRR_OPT_PERSIST_WAIT_MS = 5, /* longest time a task of the persistent launch waits for its
                                  system's earlier stages (default 30000 ms); past it the
                                  launch gives up and the fit returns KRR_EDEVICE */
  KRR_OPT_GRAPHS = 6,       /* 1: krr_fit and krr_predict run their device work as HIP graph
                               replays: the second call with the same shapes, settings,
                               pointers and stream captures it (the first runs eagerly and
                               sizes the workspace), later calls replay it; krr_fit's
                               grouping, status readback and model creation stay outside
                               the graph, and refinement takes its first steps inside it
                               (device-side early exit), any further ones outside.  Results
                               are identical to 0 (default), which launches directly.
                               Setting the option drops the captured graphs */
  KRR_OPT_AUTOTUNE = 7,     /* 1 (default): every system takes the panel width krr_autotune
                               recorded for its precision and size class (the default width
                               where none is recorded); a batch whose systems then differ in
                               width is factored by the persistent launch; 0: every system
                               takes KRR_OPT_PANEL_TILES */
  KRR_OPT_FACTOR_STREAMS = 8 /* 1..4 (default 2): the launch-sequence factorisation splits the
                               batch into this many groups of consecutive systems (of about
                               equal work, at least 8 systems each) and factors them at the
                               same time on as many streams, so that one group's
                               latency-bound launches leave room for the others'; results are
                               identical for every value */,
  KRR_OPT_COLUMN_PAIRS = 9  /* 1 (default): the mixed-precision launch sequence updates two
                               panel columns per launch in one pass over each tile row's
                               packed operands (the diagonal blocks two columns ahead); 0: one
                               column per launch.  Results are identical bit for bit */
} krr_option;

/* ---- autotuning (Cholesky panel width) ------------------------------------
 * Times fits of n_sys synthetic, well-conditioned systems of m points in d
 * dimensions at precision prec (krr_prec) for a set of panel widths (2 .. 64
 * tiles, at most the system's tile rows), and records the fastest for the
 * size class of m (tile rows rounded up to a power of two) and prec on the
 * context; later fits give each system the width of its own class (see
 * KRR_OPT_AUTOTUNE), so a system's result does not depend on the batch.  If
 * the environment variable KRR_TUNE_CACHE names a file, the record is
 * appended to it ("prec class width ms" per line) and contexts created later
 * read it.  *panel_out (host) receives the width, *ms_out (host, nullable)
 * the median fit time in ms.  Synchronises `stream`; uses the context's
 * workspace (n_sys m (d + 2) x 4 bytes of trial data besides the fits'). */
krr_status krr_autotune(krr_ctx ctx, hipStream_t stream, int32_t prec, int64_t m, int32_t d, int32_t n_sys,
                        int32_t* panel_out, double* ms_out);

/* ---- context ------------------------------------------------------------
 * krr_create: bind a context to `device` (HIP ordinal).  hbm_budget_bytes
 * caps the device memory the context's workspace and models may hold
 * (0 = no cap); calls that would exceed it return KRR_EBUDGET before
 * allocating.  *out receives the handle.
 * krr_destroy: frees the workspace; models created on the context must be
 * freed first (KRR_ESTATE otherwise).  krr_last_error: message of the last
 * failing call ("" if none); the string lives until the next call. */
krr_status  krr_create(int device, size_t hbm_budget_bytes, krr_ctx* out);
krr_status  krr_destroy(krr_ctx ctx);
const char* krr_last_error(krr_ctx ctx);
krr_status  krr_set_option(krr_ctx ctx, int32_t option, int64_t value);
/* Bytes of device memory currently held by the context (workspace + models +
 * released model blocks kept for reuse by later models of the same size). */
krr_status  krr_memory_in_use(krr_ctx ctx, size_t* bytes);
/* Graphs captured and graph replays launched on the context (KRR_OPT_GRAPHS;
 * host outputs). */
krr_status  krr_graph_counts(krr_ctx ctx, int64_t* captured, int64_t* replayed);
/* Timing record of the launches made since timing was enabled or last
 * reported: synchronises the device and writes a NUL-terminated JSON object
 * {"<kernel class>": {"count": launches, "ms": summed event time, "busy_ms":
 * time covered by at least one of the class's launches (launches on several
 * streams overlap), "flops": summed algorithmic flops, "bytes": summed
 * algorithmic bytes}, ...} into buf (host, cap bytes, truncated if short);
 * the class "chol" unites the intervals of all "chol_*" classes (the
 * factorisation's wall time).  *needed (host, nullable) receives the full length including the
 * NUL.  The record is cleared when buf is given; buf = NULL only queries the
 * length. */
krr_status  krr_timing_report(krr_ctx ctx, char* buf, size_t cap, size_t* needed);

/* ---- sparse input (Section 5.5; Section 6) ---------------------------------
 * Expands an n x d matrix held in CSR form into the dense row-major matrix
 * that krr_partition, krr_fit, krr_predict and krr_select take.
 * indptr:  device, n + 1 int64 row pointers: row i holds the entries
 *          k in [indptr[i], indptr[i + 1]); indptr[0] = 0, non-decreasing,
 *          indptr[n] = nnz.
 * indices: device, nnz int32 column indices in [0, d), any order; a column
 *          repeated in a row is summed (storage order, in dtype).
 * values:  device, nnz values of dtype `dtype` (KRR_F32 / KRR_F64).
 * X:       device, n x d output of the same dtype, fully overwritten.
 * indices and values may be NULL when nnz = 0.  Synchronises `stream` to
 * check the structure: a malformed one returns KRR_EINVAL (X then holds
 * zeros in the malformed rows and entries, the other rows expanded). */
krr_status krr_csr_to_dense(krr_ctx ctx, hipStream_t stream, const int64_t* indptr, const int32_t* indices,
                            const void* values, int32_t dtype, int64_t n, int32_t d, int64_t nnz, void* X);

/* ---- partition (Section 2.4 Algorithm 2; Section 4.3 Algorithm 4) --------
 * X:         device, n x d row-major, dtype `dtype` (FP32 values are widened
 *            exactly to FP64 for every distance).
 * p:         number of partitions (1 <= p <= n, p <= 1024).
 * method:    krr_part.  lloyd_iters: maximum Lloyd passes (KMEANS, KBALANCE,
 *            KBALANCE_APPROX); a pass with no changed assignment ends the
 *            loop early.
 * seed:      SplitMix64 seed of the k-means++ draws.
 * centroids: device, p x d FP64; input for GIVEN, output otherwise.
 * assign:    device, n int32 output: partition of each point.  For KMEANS and
 *            GIVEN the nearest centre (squared FP64 distance, summed in feature
 *            order without fused multiply-add, lowest index on ties); for
 *            KBALANCE the greedy capacity-constrained choice.
 * sizes:     device, p int64 output: points per partition.
 * Asynchronous. */
krr_status krr_partition(krr_ctx ctx, hipStream_t stream,
                         const void* X, int32_t dtype, int64_t n, int32_t d,
                         int32_t p, int32_t method, int32_t lloyd_iters, uint64_t seed,
                         double* centroids, int32_t* assign, int64_t* sizes);

/* ---- fit (Section 2.3 Eq. 6, Algorithm 1 per partition; Algorithm 5) -----
 * X, y:      device, n x d and n, both of dtype `dtype`.
 * assign:    device, n int32 in [0, p): partition of each point.
 * centroids: device, p x d FP64 (kept in the models for routing).
 * params:    host, n_params settings (1 <= n_params <= 4096,
 *            n_params * p <= 65535), all fitted in one batch of
 *            n_params * p systems (K_j + lambda I) alpha_j = y_j; all
 *            settings of a call share the precision.
 * models_out: host array of n_params handles (one model per setting).
 * info_out:  host array of n_params * p records, index param * p + j.
 * Synchronises `stream`.  Returns KRR_ENOTSPD / KRR_ENOCONV if any system
 * failed (its info record says which; the other systems' results stay
 * valid and every model is still created), KRR_EBUDGET if the factor
 * storage would exceed the budget.  Models copy what they need from X, y, so
 * the caller may free them once the call returns. */
krr_status krr_fit(krr_ctx ctx, hipStream_t stream,
                   const void* X, const void* y, int32_t dtype, int64_t n, int32_t d,
                   const int32_t* assign, const double* centroids, int32_t p,
                   const krr_fit_params* params, int32_t n_params,
                   krr_model* models_out, krr_part_info* info_out);

/* ---- predict (Eq. 7; Sections 4.1, 4.2; Algorithm 5) ---------------------
 * Xt:        device, k x d of dtype `dtype`.
 * yhat:      device FP64 output: k values (NEAREST, AVERAGE) or k x p
 *            row-major (ALL).
 * route_out: device k int32 output (nearest centre), may be NULL.
 * Asynchronous.  Predictions are evaluated in FP64 for every precision. */
krr_status krr_predict(krr_ctx ctx, hipStream_t stream, krr_model model,
                       const void* Xt, int32_t dtype, int64_t k, int32_t route,
                       double* yhat, int32_t* route_out);

/* ---- predict without device allocation -------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, routes and result as krr_predict (the same kernels with the same
 * launch shapes, so the values are identical bit for bit), but every
 * temporary buffer of the call (routes, grouping counts, partial sums, the
 * per-model matrix of AVERAGE) is carved from a fixed device array of
 * KRR_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends; the call allocates and frees no device memory and
 * records no timing events.  A call whose temporaries would not fit returns
 * KRR_EINVAL before any work is queued, with the bytes it needs in
 * krr_last_error (NEAREST fits roughly k <= 250,000 points; ALL and AVERAGE
 * roughly k * p <= 250,000).  Every call on one GPU shares the array, which
 * keeps the last call's contents (no temporary needs to start at zero):
 * calls that overlap on one GPU -- other streams, other contexts, other host
 * threads -- race, and the caller must order them.  Asynchronous. */
#define KRR_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
krr_status krr_predict_noalloc(krr_ctx ctx, hipStream_t stream, krr_model model,
                               const void* Xt, int32_t dtype, int64_t k, int32_t route,
                               double* yhat, int32_t* route_out);

/* ---- select (Eq. 3; Algorithm 5 model choice) ----------------------------
 * Predicts the k validation points Xv with every model, mse_out[i] =
 * mean((yhat_i - yv)^2) (host, n_models), *best_out = index of the lowest MSE
 * (strict "<": the first model wins ties; host).  route: NEAREST, AVERAGE or
 * LABEL (yhat_i per point = the partition model closest to its label, i.e.
 * the squared error is the minimum over the p models; Algorithm 6); ALL is
 * rejected with KRR_EINVAL.  Synchronises `stream`. */
krr_status krr_select(krr_ctx ctx, hipStream_t stream,
                      const krr_model* models, int32_t n_models,
                      const void* Xv, const void* yv, int32_t dtype, int64_t k, int32_t route,
                      double* mse_out, int32_t* best_out);

/* ---- models ---------------------------------------------------------------
 * krr_model_alpha: copy alpha of partition j (m_j FP64 values, in the order
 * of increasing original point index within the partition) to device memory
 * `alpha` (asynchronous on `stream`); *m receives m_j (host).
 * krr_model_free: release a model (NULL is accepted); waits for the work its
 * context has queued (on every stream the context has used; other contexts'
 * work is not waited for), then keeps the model's memory in its context for
 * reuse by later models (see krr_memory_in_use; freed by krr_destroy or under
 * budget pressure). */
krr_status krr_model_alpha(krr_ctx ctx, hipStream_t stream, krr_model model, int32_t j,
                           double* alpha, int64_t* m);
krr_status krr_model_free(krr_model model);

/* ---- serving: continuous batching over a resident model ------------------
 * A server keeps one fitted model resident (typically the p partition models
 * of Algorithm 5 for one setting) and answers two kinds of request from
 * host memory:
 *   predict: k query points routed to the nearest centre's model (KKRR2 /
 *            BKRR2, Section 4.2, Algorithm 5) and evaluated with Eq. 7;
 *   fit:     an independent problem (K + lambda I) alpha = y of m points
 *            (Eq. 6, Algorithm 1), returned as alpha.
 * Requests queue per kind.  Worker threads, each with its own context and
 * stream, take a batch whenever they are idle: a predict worker takes the
 * queued predict requests in arrival order (at most max_batch_points points)
 * and serves them with one routed prediction; a fit worker takes the oldest
 * fit request and every later queued one with the same d and settings (at
 * most max_batch_fits) and solves them as one ragged batch, one partition
 * per request.  A request is admitted into a batch only while the estimated
 * device memory of all admitted, unfinished requests stays within
 * hbm_budget_bytes, so requests that arrive while others run wait until
 * memory and a worker free up; batches of different workers run
 * concurrently on the device.  A request's result depends only on its own
 * data (the batch it joins changes no arithmetic of a fit, and only the
 * summation split of a prediction).  Latency of a request = time from its
 * submit call to the end of the batch that served it.  Every worker has its
 * own stream; for predict batches not to queue behind fit kernels the process
 * needs a hardware queue per stream (HIP's GPU_MAX_HW_QUEUES, default 4, set
 * before the runtime starts, at least workers + 1). */
typedef struct krr_server_s* krr_server;

typedef struct {
  int32_t predict_workers;   /* >= 1 */
  int32_t fit_workers;       /* >= 0 (0: fit requests are rejected) */
  int32_t max_batch_fits;    /* >= 1: fit requests per batch */
  int32_t reserved;          /* must be 0 */
  int64_t max_batch_points;  /* >= 1: query points per predict batch */
  size_t  hbm_budget_bytes;  /* device memory of the serving workers together (0 = none):
                                split into 2 x the estimate of a full predict batch per
                                predict worker and equal shares of the rest per fit
                                worker; admission keeps the estimated memory of
                                unfinished requests within it, and a fit request above
                                one fit worker's share is rejected (KRR_EBUDGET) */
} krr_server_config;

typedef struct {
  int32_t status;            /* KRR_OK or the error of the request's batch / system */
  int32_t kind;              /* 0 predict, 1 fit */
  int32_t batch_requests;    /* requests in the batch that served it */
  int32_t reserved;
  double  queue_ms;          /* submit -> batch start */
  double  run_ms;            /* batch start -> batch end */
  double  total_ms;          /* submit -> batch end */
} krr_request_info;

typedef struct {
  int64_t predict_requests;  /* completed since creation or the last reset */
  int64_t fit_requests;
  int64_t points;            /* query points predicted */
  int64_t fit_rows;          /* training points fitted */
  int64_t predict_batches;
  int64_t fit_batches;
  int64_t failed;            /* completed requests with a status other than KRR_OK */
  int64_t max_inflight_bytes;/* peak estimated memory of admitted, unfinished requests */
  int64_t max_device_bytes;  /* peak device memory held by the workers' contexts together
                                (measured after each batch; at most hbm_budget_bytes) */
  double  predict_p50_ms, predict_p99_ms;   /* nearest-rank percentiles of total_ms */
  double  fit_p50_ms, fit_p99_ms;
  double  span_ms;           /* first submit -> last completion */
} krr_serve_stats;

/* krr_server_create: start a server on the device of `owner` that answers
 * predict requests with `model` (created on `owner`, whose dimension d fixes
 * the query width).  The model and owner must outlive the server, and the
 * owner context must not free the model meanwhile; the server itself never
 * uses the owner context.  *out receives the handle.
 * krr_server_destroy: waits for every submitted request, stops the workers
 * and frees their contexts.  Results of requests not yet waited for stay
 * written to their host buffers; their tickets are dropped. */
krr_status  krr_server_create(krr_ctx owner, krr_model model, const krr_server_config* cfg,
                              krr_server* out);
krr_status  krr_server_destroy(krr_server server);
/* Message of the last failing server call or request ("" if none). */
const char* krr_server_last_error(krr_server server);

/* Submit requests (thread-safe; returns at once).  Host buffers are owned by
 * the caller and must stay valid until krr_server_wait returns for the ticket.
 * predict: Xq host FP32 k x d (d of the resident model), yhat host FP64 k out.
 * fit:     X host FP32 m x d, y host FP32 m, params host (one setting),
 *          alpha host FP64 m out (in the order of the m points).
 * *ticket receives the request's id.  KRR_EINVAL for bad sizes or null
 * pointers; KRR_EBUDGET if the request alone would exceed the budget;
 * KRR_ESTATE if the server has no fit workers (fit) or is stopping. */
krr_status  krr_server_submit_predict(krr_server server, const float* Xq, int64_t k, double* yhat,
                                      int64_t* ticket);
krr_status  krr_server_submit_fit(krr_server server, const float* X, const float* y, int64_t m,
                                  int32_t d, const krr_fit_params* params, double* alpha,
                                  int64_t* ticket);
/* Block until the request is done; *info (host, nullable) receives its record.
 * Returns the request's status; the ticket is released (KRR_EINVAL if unknown). */
krr_status  krr_server_wait(krr_server server, int64_t ticket, krr_request_info* info);
/* Counters and latency percentiles of completed requests (host out); reset = 1
 * clears them after reading. */
krr_status  krr_server_stats(krr_server server, int32_t reset, krr_serve_stats* out);

#ifdef __cplusplus
}
#endif
#endif /* KRR_H_ */
