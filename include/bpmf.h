/*
 * bpmf.h -- C ABI of the MI355X (gfx950) BPMF Gibbs row-update library.
 *
 * The method: Bayesian probabilistic matrix factorisation sampled with Gibbs
 * sweeps (paper: Section 2 "BPMF" and Algorithm 1).  The rating matrix R
 * (M users x N movies, very sparse) is approximated by U V^T with U (M x K)
 * and V (N x K) (Section 1).  Every sweep draws the hyper-parameters of one
 * side from that side's factor matrix, then redraws every row of that side
 * from its Gaussian conditional given the other side and its ratings, then
 * does the same for the other side, then predicts the test points.  The row
 * draw builds the K x K precision from the prior plus the outer products of
 * the rated items' factor rows and factors it with a Cholesky decomposition
 * instead of inverting it, because it is used only once (Section 3.1).
 *
 * Conventions of this library (the paper prints no formula):
 *   row i:  P = Lambda + alpha sum_{j in Omega_i} v_j v_j^T,
 *           b = Lambda mu + alpha sum_{j in Omega_i} (r_ij - rbar) v_j,
 *           L L^T = P (lower, positive diagonal), x_i = L^{-T}(L^{-1} b + z_i)
 *   side:   (mu, Lambda) ~ Normal-Wishart posterior with xbar, centred scatter
 *           S, beta* = beta0 + n, nu* = nu0 + n, mu* = (beta0 mu0 + n xbar)/beta*,
 *           W*^{-1} = W0^{-1} + S + beta0 n / beta* (xbar - mu0)(xbar - mu0)^T,
 *           Lambda = L_W A A^T L_W^T (Bartlett, L_W = chol(W*)),
 *           mu = mu* + chol(beta* Lambda)^{-T} z.
 *   sweep:  users' half first, then movies'; hypers of a side come from that
 *           side's current matrix.
 *
 * Memory: every pointer named d_* is device memory owned by the caller, who
 * keeps it alive for the lifetime of the context that uses it.  The library
 * allocates no device memory for a sampler: scratch comes from the caller's
 * workspace (size from bpmf_workspace_size).  Host pointers (h_*, and the
 * mu0 / W0 members of bpmf_params) are read during the call only.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the legacy
 * default stream).  Calls enqueue work and return; results are ready when
 * the stream is synchronised, unless stated otherwise.
 *
 * Errors: every function returns a bpmf_status and never aborts or throws.
 * bpmf_last_error() gives a thread-local message for the last failure.
 * Invalid arguments are rejected before any device work is enqueued.
 */
#ifndef BPMF_H
#define BPMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BPMF_OK = 0,
    BPMF_E_INVALID = 1,   /* bad argument: shapes, pointers, CSR/CSC structure, parameters */
    BPMF_E_NOT_SPD = 2,   /* W0 (or a stored precision) is not symmetric positive definite */
    BPMF_E_WORKSPACE = 3, /* workspace missing or smaller than required */
    BPMF_E_STATE = 4,     /* context unusable (NULL, destroyed, or a previous fatal error) */
    BPMF_E_HIP = 5,       /* a HIP runtime call or kernel launch failed */
    BPMF_E_NOMEM = 6      /* host allocation failed */
} bpmf_status;

/* Arithmetic of the row update.
 *   BPMF_FP64: everything in FP64; U and V are double.
 *   BPMF_FP32: FP32 gathers, FP32 Gram on matrix cores, FP32 Cholesky; U, V float.
 *   BPMF_BF16: BF16 copies of U and V are gathered; Gram on BF16 matrix cores
 *              with FP32 accumulation; FP32 Cholesky; U, V float.
 * In FP32/BF16 a row whose FP32 Cholesky pivot is not finite or falls below
 * 64 K 2^-24 max_k P_kk is recomputed from the FP32 factors in FP64.
 * The hyper-parameter step is always FP64. */
typedef enum { BPMF_FP64 = 0, BPMF_FP32 = 1, BPMF_BF16 = 2 } bpmf_precision;

/* Rating matrix in both orientations (Section 1: R is M x N, sparse).
 * CSR: row_ptr[M+1] (int64, row_ptr[0] = 0, nondecreasing, row_ptr[M] = nnz),
 *      col_idx[nnz] (int32, strictly increasing within a row, in [0, N)),
 *      row_val[nnz].
 * CSC: the same matrix by columns: col_ptr[N+1], row_idx[nnz], col_val[nnz].
 * All device pointers.  val_is_f64 = 1: values are double, 0: float. */
typedef struct {
    int64_t M, N, nnz;
    const int64_t *d_row_ptr;
    const int32_t *d_col_idx;
    const void *d_row_val;
    const int64_t *d_col_ptr;
    const int32_t *d_row_idx;
    const void *d_col_val;
    int32_t val_is_f64;
} bpmf_ratings;

/* Launch shape of the mixed-precision sweep (FP32/BF16 modes, K <= 64):
 * how the rating-count-ordered row table is cut into launches.  Rows are
 * independent given the hyper-parameters (Section 3.1), so every shape samples
 * the same conditional; shapes differ only in summation order (pieces of a
 * heavy row are summed piece by piece) and in whether a row with few ratings
 * takes rank-one updates of chol(Lambda) instead of a fresh factorisation
 * (Section 3.1), i.e. within FP32 rounding.  A field of 0 keeps the built-in
 * choice.  Read once by bpmf_init; ignored in BPMF_FP64 and for K > 64.
 *   heavy_min_ratings  rows with at least this many ratings are cut into
 *                      pieces (0: 2048; else >= 64)
 *   piece_min_ratings  shortest piece (0: 512; else >= 64)
 *   heavy_split        1: always cut heavy rows, -1: never, 0: only when they
 *                      hold >= 10% of the ratings
 *   rank1_max_ratings  rows with at most this many ratings take the rank-one
 *                      kernels (0: 3 for K <= 32, 2 for K <= 64; -1: none;
 *                      else 1..4)
 *   rank1_split        1: always use the rank-one launch when such rows exist,
 *                      -1: never, 0: only when they are >= 16384 rows or
 *                      >= 1/16 of the side
 *   kernel_variant     code variant of the one-wavefront row kernel at
 *                      32 < K <= 64 (the same arithmetic, other rounding order
 *                      or register budget): 0 or 1: the Cholesky's trailing
 *                      updates beyond the next panel on FP32 matrix cores,
 *                      4 wavefronts per SIMD; 2: those updates on the vector
 *                      units within each 32-column half; 3: as 1, register
 *                      allocation held to 3 wavefronts per SIMD
 * Out-of-range fields make bpmf_workspace_size and bpmf_init return
 * BPMF_E_INVALID. */
typedef struct {
    int32_t heavy_min_ratings;
    int32_t piece_min_ratings;
    int32_t heavy_split;
    int32_t rank1_max_ratings;
    int32_t rank1_split;
    int32_t kernel_variant;
} bpmf_launch_shape;

/* Model and run parameters (Section 2: Gaussian rows, Normal-Wishart hyperpriors).
 *   K          latent dimension, 1..128
 *   precision  bpmf_precision
 *   alpha      rating precision, > 0 (fixed, not sampled)
 *   beta0      > 0; nu0 > K - 1; mu0[K] and W0[K*K] (row-major, SPD) host pointers
 *   mean_rating  rbar subtracted from ratings and added to predictions;
 *                NaN = the FP64 mean of the stored values (computed at init)
 *   seed       key of the device counter-based generator (Philox4x32-10)
 *   burnin     sweeps before test predictions are averaged
 *   use_graph  1 = replay whole sweeps from a captured HIP graph (Philox mode)
 *   validate   1 = copy CSR/CSC to the host at init and check the structure
 *              (monotone pointers, sorted unique in-range indices, CSR == CSC)
 *   shape      optional launch shape (host pointer, NULL = built-in choices),
 *              read during the call */
typedef struct {
    int32_t K;
    int32_t precision;
    double alpha;
    double beta0;
    double nu0;
    const double *mu0;
    const double *W0;
    double mean_rating;
    uint64_t seed;
    int32_t burnin;
    int32_t use_graph;
    int32_t validate;
    const bpmf_launch_shape *shape;
} bpmf_params;

typedef struct bpmf_ctx bpmf_ctx;

/* Bytes of device workspace bpmf_init needs for this problem (including the
 * running sums of n_test held-out predictions). */
bpmf_status bpmf_workspace_size(const bpmf_ratings *R, const bpmf_params *p, int64_t n_test,
                                size_t *bytes);

/* Creates a sampler.  d_U (M x K) and d_V (N x K), row-major, hold the initial
 * state and always the current sample afterwards: double in BPMF_FP64, float
 * otherwise.  d_ws is the caller's workspace of ws_bytes.  n_test held-out
 * pairs (d_test_rows, d_test_cols, int32, device) get a running mean of their
 * predictions over sweeps >= burnin.  Errors: BPMF_E_INVALID (shapes, ranges,
 * CSR/CSC structure when validate = 1; BPMF_BF16 also needs M, N < 2^24), BPMF_E_NOT_SPD (W0),
 * BPMF_E_WORKSPACE, BPMF_E_HIP.  Synchronises `stream` before returning. */
bpmf_status bpmf_init(bpmf_ctx **ctx, const bpmf_ratings *R, const bpmf_params *p, void *d_U,
                      void *d_V, void *d_ws, size_t ws_bytes, int64_t n_test,
                      const int32_t *d_test_rows, const int32_t *d_test_cols, void *stream);

/* Runs n_sweeps Gibbs sweeps (Algorithm 1).  d_tape = NULL: draws come from
 * the device counter-based generator keyed by (seed, sweep, side, row).
 * Otherwise d_tape (device, double) holds the draws of exactly these sweeps:
 * per half-sweep over n rows (users' half first) K chi-square draws with
 * nu0 + n - k degrees of freedom (k = 0..K-1), K(K-1)/2 Bartlett normals
 * (row-major strict lower part), K mean normals, then n*K row normals
 * (row-major); tape_len must equal n_sweeps times that count for both halves.
 * Errors: BPMF_E_STATE, BPMF_E_INVALID (tape length), BPMF_E_HIP. */
bpmf_status bpmf_sweep(bpmf_ctx *ctx, int32_t n_sweeps, const double *d_tape, int64_t tape_len,
                       void *stream);

/* Algorithm 1's prediction step for arbitrary pairs: predictions
 * u_i . v_j + rbar of the current sample for n pairs (device
 * int32 rows/cols, device double output).  Errors: BPMF_E_INVALID if n < 0 or
 * pointers are NULL with n > 0 (indices are range-checked only when
 * validate = 1, on the host). */
bpmf_status bpmf_predict(bpmf_ctx *ctx, int64_t n, const int32_t *d_rows, const int32_t *d_cols,
                         double *d_out, void *stream);

/* Running posterior-mean predictions of the held-out pairs given at init
 * (device double[n_test]); *h_count (host) receives how many sweeps entered
 * the mean.  Synchronises `stream`. */
bpmf_status bpmf_test_predictions(bpmf_ctx *ctx, double *d_mean, int64_t *h_count, void *stream);

/* Current hyper-parameters, synchronously copied to host memory:
 * h_out[2 K^2 + 2 K] = [Lambda_U (K x K), mu_U, Lambda_V (K x K), mu_V], FP64. */
bpmf_status bpmf_get_hyper(bpmf_ctx *ctx, double *h_out, void *stream);

typedef struct {
    int64_t sweeps_done;
    int64_t fallback_rows; /* rows recomputed in FP64 since init (FP32/BF16 modes) */
    int64_t nonfinite_rows;/* rows whose FP64 draw was not finite since init */
    double mean_rating;
    int32_t K, precision;
    /* how init cut each side's rows into launches (users [0], movies [1]):
     * rows taken by the rank-one kernels, heavy rows cut into pieces and
     * their piece count; the other rows run in the one-wavefront launch
     * (FP32/BF16 with K <= 64; zero otherwise) */
    int64_t rank1_rows[2], heavy_rows[2], pieces[2];
    int32_t kernel_variant; /* resolved bpmf_launch_shape::kernel_variant (0: none applies) */
} bpmf_info;

/* Counters; synchronises `stream`. */
bpmf_status bpmf_get_info(bpmf_ctx *ctx, bpmf_info *info, void *stream);

/* Serving support (not a step of the paper's sampler): keeps a posterior
 * sample for folding in new users.  Copies the current movie factors (as
 * float, N x K) and the user-side hyper-parameters (Lambda_U as double
 * K x K, mu_U as double K) into a caller-owned fold-in sample slot (device
 * pointers); S such slots, taken a sweep or more apart, form the
 * bpmf_foldin_model of the fold-in functions below.  Errors: BPMF_E_STATE,
 * BPMF_E_INVALID (NULL slot), BPMF_E_HIP. */
bpmf_status bpmf_snapshot(bpmf_ctx *ctx, float *d_V_slot, double *d_Lambda_slot,
                          double *d_mu_slot, void *stream);

/* Saved sampler state: sweep counter, U, V, hypers and prediction sums.
 * bpmf_state_size gives the bytes; save/restore use host memory and
 * synchronise `stream`.  A restored context continues bit-identically. */
bpmf_status bpmf_state_size(bpmf_ctx *ctx, size_t *bytes);
bpmf_status bpmf_state_save(bpmf_ctx *ctx, void *h_buf, size_t bytes, void *stream);
bpmf_status bpmf_state_restore(bpmf_ctx *ctx, const void *h_buf, size_t bytes, void *stream);

/* Per-kernel timing.  While enabled, sweeps run eagerly (no graph replay) and
 * every launch is bracketed by HIP events recorded on the launch stream;
 * bpmf_get_timing synchronises, resolves the pending events and returns the
 * accumulated milliseconds and launch counts per kernel class:
 * [0] side statistics, [1] hyper-parameter step, [2] users' row update,
 * [3] movies' row update, [4] FP64 recompute of flagged rows,
 * [5] predictions, [6] sweep counter, [7] rank-one row update of rows with
 * very few ratings, [8] factorisation of rows with very many ratings, whose
 * Gram was computed in pieces within [2] / [3] (both sides; [7] and [8]
 * FP32/BF16 with K <= 64). */
#define BPMF_TIMING_CLASSES 9
typedef struct {
    double ms[BPMF_TIMING_CLASSES];
    int64_t launches[BPMF_TIMING_CLASSES];
} bpmf_timing;
bpmf_status bpmf_set_timing(bpmf_ctx *ctx, int32_t enable);
bpmf_status bpmf_get_timing(bpmf_ctx *ctx, bpmf_timing *out, int32_t reset);

/* Releases the context (host objects and graphs only). NULL is ignored. */
bpmf_status bpmf_destroy(bpmf_ctx *ctx);

/* ------------------------------------------------------------------------ */
/* Fold-in: conditional means of new users against stored posterior samples */
/* ------------------------------------------------------------------------ */

/* S stored samples of the movie factors and the user hypers:
 *   d_V[S][N][K] float, d_Lambda[S][K][K] double (SPD), d_mu[S][K] double. */
typedef struct {
    int32_t S, K;
    int64_t N;
    double alpha;
    double mean_rating;
    const float *d_V;
    const double *d_Lambda;
    const double *d_mu;
} bpmf_foldin_model;

/* Bytes of workspace bpmf_foldin needs for a batch with n_queries query
 * columns in total (S * n_queries floats of per-sample partial predictions). */
bpmf_status bpmf_foldin_workspace_size(const bpmf_foldin_model *m, int64_t n_queries,
                                       size_t *bytes);

/* Fold-in of new users (serving; the paper's row conditional of Section 2
 * with z = 0, averaged over stored posterior samples, not a step of its
 * sampler).  For each request r (ratings d_cols/d_vals[d_req_ptr[r] .. d_req_ptr[r+1]),
 * query columns d_q_cols[d_q_ptr[r] .. d_q_ptr[r+1]), d_q_ptr[n_req] =
 * n_queries) and each sample s:
 *   m_s = (Lambda_s + alpha sum_j v_j v_j^T)^{-1}(Lambda_s mu_s + alpha sum_j (r_j - rbar) v_j)
 * with v_j rows of sample s, and d_out[q] = rbar + (1/S) sum_s m_s . v_q (FP32
 * arithmetic, samples summed in order).  Stateless: calls on different
 * streams with different workspaces may overlap.  Each request's result does
 * not depend on the other requests in the batch.  Errors: BPMF_E_INVALID,
 * BPMF_E_WORKSPACE, BPMF_E_HIP.  K must be <= 64.  A (request, sample) pair
 * whose FP32 Cholesky pivot is not finite or not above 64 K 2^-24 max_k P_kk
 * is recomputed in FP64 (Gram of the FP32 sample rows, Cholesky and solves in
 * FP64) before the average over samples; only a pivot that fails in FP64 too
 * (a model that is not SPD) gives NaN predictions. */
bpmf_status bpmf_foldin(const bpmf_foldin_model *m, int64_t n_req, const int64_t *d_req_ptr,
                        const int32_t *d_cols, const float *d_vals, const int64_t *d_q_ptr,
                        const int32_t *d_q_cols, int64_t n_queries, float *d_out, void *d_ws,
                        size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as bpmf_foldin, with the per-sample partial
 * predictions kept in a library-owned device array instead of a caller
 * workspace.  The array holds bpmf_foldin_noalloc_max_partials() floats
 * (4 MiB; S * n_queries must not exceed it, else BPMF_E_INVALID before any
 * device work); each GPU the library runs on has its own copy, held until
 * the process ends, found on the first call on that device.  The call itself
 * allocates nothing: no hipMalloc, hipFree or allocating library routine.
 * Every call on one GPU uses that GPU's array and leaves its contents there;
 * nothing in it has to start at zero.  Calls that overlap on one GPU (on
 * streams not ordered with each other, or from several threads) race on the
 * array; order them.  Errors: BPMF_E_INVALID, BPMF_E_HIP. */
bpmf_status bpmf_foldin_noalloc(const bpmf_foldin_model *m, int64_t n_req, const int64_t *d_req_ptr,
                                const int32_t *d_cols, const float *d_vals, const int64_t *d_q_ptr,
                                const int32_t *d_q_cols, int64_t n_queries, float *d_out, void *stream);
int64_t bpmf_foldin_noalloc_max_partials(void);

/* ------------------------------------------------------------------------ */
/* Fold-in serving engine: continuous batching on several streams             */
/* ------------------------------------------------------------------------ */

/* A server owns device buffers and pinned staging for n_streams batches in
 * flight, sized so that all of them together stay within mem_budget_bytes,
 * and a dispatcher thread.  Requests are queued by bpmf_server_submit (host
 * arrays are copied; any thread).  Whenever a stream is free, the dispatcher
 * takes queued requests in arrival order while the batch fits the stream's
 * share of the budget, at most max_batch requests per batch and at most
 * max_inflight requests on the GPU in total, uploads the batch, runs
 * bpmf_foldin on it and downloads the predictions; batches on different
 * streams overlap.  A request never waits for a batch to fill: a free stream
 * takes what is queued.  Results are identical to serving the request alone
 * (bpmf_foldin computes each request independently).
 * The model arrays must stay alive and unchanged while the server exists. */
typedef struct bpmf_server bpmf_server;

typedef struct {
    int64_t requests_done;
    int64_t batches;
    int64_t max_batch;        /* largest batch launched */
    int64_t max_inflight;     /* most requests on the GPU at once */
    int64_t max_batch_bytes;  /* largest batch footprint in device memory */
    int64_t stream_capacity;  /* bytes available to one batch */
} bpmf_server_stats;

/* Errors: BPMF_E_INVALID (model, n_streams < 1, budget too small for one
 * request of one rating and one query), BPMF_E_HIP, BPMF_E_NOMEM. */
bpmf_status bpmf_server_create(bpmf_server **srv, const bpmf_foldin_model *m,
                               size_t mem_budget_bytes, int32_t n_streams, int32_t max_batch,
                               int32_t max_inflight);

/* Resident mode: no launch and no host-issued copy per request.  One
 * persistent kernel owns n_slots request slots (at most max_nnz ratings and
 * max_q queries each) in coherent pinned
 * host memory; the dispatcher writes a queued request into a free slot, the
 * kernel computes it (one workgroup per slot, one wavefront in it per stored
 * sample, the same arithmetic as bpmf_foldin, so the same predictions) and
 * writes the predictions back.  The resident kernel has no FP64 path: a
 * request with a (request, sample) pair whose FP32 pivot fails is computed
 * again by bpmf_foldin on a stream of the server, which recomputes that pair
 * in FP64, so predictions equal batching mode's in that case too.  A request's samples share one compute unit,
 * so large requests take longer than in batching mode, which spreads them.
 * The kernel ends after idle_polls polls without a request (0: 500000, about
 * a second) or when the server is destroyed, and is launched again when a
 * request waits.  submit / poll / drain / replay / stats / destroy work as in
 * batching mode; stats count each request as a batch of one.
 * Errors: BPMF_E_INVALID (model with S > 16 or K > 64, n_slots outside
 * 1..256 or above the slot workgroups the device holds at once, max_nnz
 * outside 1..2^20, max_q outside 1..1024), BPMF_E_HIP. */
bpmf_status bpmf_server_create_resident(bpmf_server **srv, const bpmf_foldin_model *m, int32_t n_slots,
                                        int32_t max_nnz, int32_t max_q, int64_t idle_polls);

/* Queues one request (host arrays: nnz column indices in [0, N) and ratings,
 * nq query columns in [0, N)).  BPMF_E_INVALID if an index is out of range or
 * the request alone exceeds one stream's share of the budget (resident mode:
 * the slot size). */
bpmf_status bpmf_server_submit(bpmf_server *srv, int64_t id, int32_t nnz, const int32_t *h_cols,
                               const float *h_vals, int32_t nq, const int32_t *h_q_cols);

/* Moves up to max_results finished requests out of the server: ids[i], the
 * predictions of request i at h_preds[offsets[i] .. offsets[i+1]) (offsets
 * has max_results + 1 entries, h_preds room for pred_capacity floats) and its
 * latency in seconds from submit to the host seeing the result.  *n_out
 * receives the number of results moved. Never blocks. */
bpmf_status bpmf_server_poll(bpmf_server *srv, int32_t max_results, int64_t *ids, int64_t *offsets,
                             float *h_preds, int64_t pred_capacity, double *latency_s,
                             int32_t *n_out);

/* Blocks until every submitted request has finished (results stay pollable). */
bpmf_status bpmf_server_drain(bpmf_server *srv);

bpmf_status bpmf_server_get_stats(bpmf_server *srv, bpmf_server_stats *st);

/* Real-time replay of an arrival trace: a client thread submits request i at
 * arrival_s[i] seconds after the call starts (requests in CSR form: ratings
 * h_cols/h_vals[h_ptr[i] .. h_ptr[i+1]), queries h_q_cols[h_q_ptr[i] ..
 * h_q_ptr[i+1])), then the call waits for all of them and writes each
 * request's predictions to h_out[h_q_ptr[i] ..] and its latency to
 * latency_s[i].  Requests are identified by their index. */
bpmf_status bpmf_server_replay(bpmf_server *srv, int64_t n, const double *arrival_s,
                               const int64_t *h_ptr, const int32_t *h_cols, const float *h_vals,
                               const int64_t *h_q_ptr, const int32_t *h_q_cols, float *h_out,
                               double *latency_s);

bpmf_status bpmf_server_destroy(bpmf_server *srv);

/* ------------------------------------------------------------------------ */
/* Misc                                                                      */
/* ------------------------------------------------------------------------ */
const char *bpmf_status_string(bpmf_status s);
const char *bpmf_last_error(void);
/* Library version string. */
const char *bpmf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BPMF_H */
