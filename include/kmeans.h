/*
 * kmeans.h -- C ABI of the MI355X (gfx950) mixed-precision Lloyd k-means
 * library.
 *
 * The method is that of Carson, Chen, Liu, "Computing k-means in Mixed
 * Precision": squared distances d(x,c)^2 = ||x||^2 - 2 x^T c + ||c||^2
 * (eq:dist-expanded, in its matrix form eq:dist-blas3) are evaluated with the
 * inputs quantised to a low precision (FP16 or BF16, cross term on the matrix
 * cores with FP32 accumulation); a per-pair reliability test
 * (eq:quantis-reliability-test, eq:fallback-rule-mp, Algorithm alg:mp-dist)
 * flags the pairs whose value may have lost its relative accuracy to
 * cancellation, and only those are recomputed by the direct formula
 * (x-c)^T(x-c) (eq:dist-direct) in FP64 from the original FP32 data.  Lloyd's
 * iteration (Algorithm alg:mp-kmeans) assigns each point to the nearest
 * centre and replaces each centre by the mean of its points (eq:center).
 *
 * Conventions shared by every entry point:
 *  - Points X are n x d FP32, row-major (point i is the contiguous row
 *    X[i*d .. i*d+d)); this is the paper's P = [p_1..p_n] in R^{d x n} with
 *    each column contiguous.  Centres C are k x d FP32 row-major.
 *  - Unless stated otherwise every array argument is a DEVICE pointer owned
 *    by the caller (for instance a contiguous PyTorch tensor).  Inputs and
 *    outputs must not alias.  The library never frees or keeps them.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  All work
 *    is enqueued on it; a call returns once the work is enqueued unless the
 *    KM_SYNC flag is set or a host-side `km_stats*` is passed, in which cases
 *    it returns after the stream has drained.
 *  - Argument errors are reported synchronously and nothing is enqueued.
 *    Data-dependent errors (non-finite input, FP16 overflow) are known only
 *    after the device work ran: they are returned when the call waits for the
 *    stream (KM_SYNC or stats != NULL) and stored in stats->data_status.
 *  - Nothing throws across this ABI, nothing aborts, nothing prints.
 *  - A context is used by one host thread at a time.  Its calls may use
 *    different streams: the device work of each call that uses the context's
 *    workspace is ordered after that of the previous such call on the same
 *    context (an event recorded at the end of every call, waited for on the
 *    next call's stream when the stream differs).  The server functions
 *    (kmeans_submit, kmeans_poll, kmeans_cancel) are thread-safe.
 */
#ifndef KMEANS_MI355X_H
#define KMEANS_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
enum {
  KM_OK = 0,
  KM_PENDING = 1,          /* kmeans_poll: request not finished yet          */
  KM_ERR_ARG = -1,         /* invalid argument (null, sizes, precision)      */
  KM_ERR_RANGE = -2,       /* an input overflows the low format (FP16 |v|>=65520) */
  KM_ERR_NONFINITE = -3,   /* NaN or Inf in X or C                           */
  KM_ERR_OOM = -4,         /* device allocation failed / over the HBM budget */
  KM_ERR_DEVICE = -5,      /* a HIP runtime call failed                      */
  KM_ERR_NOTFOUND = -6,    /* unknown ticket                                 */
  KM_ERR_CANCELLED = -7,   /* request cancelled                              */
  KM_ERR_UNSUPPORTED = -8  /* shape outside what the kernels support         */
};

/* ---- precision ------------------------------------------------------------ */
/* Low precision of the expanded formula (the paper's u_l). */
enum {
  KM_LOW_FP16 = 0,  /* binary16 inputs, FP32 accumulation (MFMA f16)        */
  KM_LOW_BF16 = 1,  /* bfloat16 inputs, FP32 accumulation (MFMA bf16)       */
  KM_LOW_FP32 = 2,  /* FP32 inputs, FP32 accumulation (MFMA f32)            */
  KM_EXACT64 = 3    /* no expanded formula: every pair by the FP64 direct
                       formula (the plain FP64 baseline kernel)             */
};

/* How the threshold alpha of the test  d^ > alpha (||x~||^2 + ||c~||^2)  is
 * chosen.  With gamma = gamma_{d+2}(u_l) = (d+2)u_l / (1-(d+2)u_l):          */
enum {
  KM_ALPHA_PAPER_EQ = 0,  /* alpha = 2 rho gamma: E^l of Section 4.3 with the
                             test eq:quantis-reliability-test (default)      */
  KM_ALPHA_PAPER_ALG = 1, /* alpha = rho gamma: the listing alg:mp-dist      */
  KM_ALPHA_EXPLICIT = 2,  /* alpha = km_precision.alpha (>= 0)               */
  KM_ALPHA_NONE = 3,      /* no fallback: uniform low-precision expanded
                             formula (the paper's "FP16"/"BF16"/"FP32" rows) */
  KM_ALPHA_HW = 4         /* alpha = rho [2 gamma_{d+2}(2^-23)
                                          + 2 (2u_l + u_l^2)(1 + u_l)^2]:
                             the error decomposition of Section 4.3
                             (arithmetic error of the expanded formula plus
                             the conversion error of the quantised inputs)
                             with the cross term accumulated in FP32 by the
                             matrix cores, whose products of FP16/BF16
                             operands are exact.  Kept pairs then have
                             relative error <= 1/(rho-1) against the exact
                             distance of the FP32 inputs.  A variant for this
                             hardware, not the paper's rule; rho > 2.      */
};
/* If (d+2) u_l >= 1 gamma is undefined and every pair is corrected. */

/* Precision u of the direct formula that replaces a flagged pair (the
 * fallback of eq:fallback-rule-mp; Section 6.1 tests the variants).  Every
 * operation is one correctly rounded operation of that format, differences
 * first, then one fused multiply-add per coordinate in index order.  The
 * refinement of the chosen label (mindist, SSE) stays FP64 in every mode. */
enum {
  KM_HIGH_FP64 = 0, /* FP64 on the FP32 inputs (default)                    */
  KM_HIGH_FP32 = 1, /* FP32 on the FP32 inputs: FP16/BF16 -> FP32           */
  KM_HIGH_LOW = 2   /* the low format itself on the quantised inputs x~, c~:
                       the uniform rule eq:fallback-rule (FP16 -> FP16,
                       BF16 -> BF16, FP32 -> FP32)                          */
};

typedef struct km_precision {
  int32_t low;        /* KM_LOW_* or KM_EXACT64                              */
  int32_t alpha_mode; /* KM_ALPHA_*                                          */
  double rho;         /* safety factor rho~ (> 2 in the paper modes; 5 by
                         default, Section 6.1)                              */
  double alpha;       /* used with KM_ALPHA_EXPLICIT only                   */
  int32_t high;       /* KM_HIGH_*; KM_EXACT64 takes KM_HIGH_FP64 only       */
  int32_t reserved;   /* zero                                                */
} km_precision;
/* A NULL km_precision* means {KM_LOW_FP16, KM_ALPHA_PAPER_EQ, 5.0, 0,
 * KM_HIGH_FP64, 0}.  A pass whose threshold flags every pair runs the direct
 * formula in the correction precision for every pair. */

typedef struct km_stats {
  int64_t n_corrected; /* pairs recomputed by the FP64 direct formula; the
                          fallback ratio eta of eq:eta is n_corrected/n_pairs */
  int64_t n_pairs;     /* pairs evaluated (n*k per assignment pass)          */
  int32_t iters;       /* Lloyd update rounds performed                      */
  int32_t data_status; /* KM_OK, KM_ERR_RANGE or KM_ERR_NONFINITE            */
  double sse_last;     /* SSE (eq:sse) of the last assignment                */
  double shift_last;   /* max_j ||c_j^t - c_j^{t-1}|| of the last update     */
  double alpha_used;   /* threshold applied (as rounded to FP32); -1 = none  */
} km_stats;

/* Flags */
#define KM_SYNC 1u        /* wait for the stream before returning */
#define KM_LABELS_HINT 2u /* kmeans_assign: labels holds an earlier assignment
                             (e.g. the previous Lloyd round); it only seeds
                             the search, the results are the same */
#define KM_ROUND_LAUNCH 4u /* kmeans_lloyd, kmeans_solve_batch: run all rounds
                              in one persistent launch where the shape allows
                              it (see kmeans_lloyd); the results are bitwise
                              the same as with one launch per phase */

typedef struct km_context km_context;
typedef struct km_server km_server;

/* One k-means problem.  In kmeans_solve_batch every pointer is a device
 * pointer; in kmeans_submit every pointer is a HOST pointer that must stay
 * valid until kmeans_poll reports completion or the request is cancelled. */
typedef struct km_problem {
  const float *X;   /* n x d points                                          */
  int64_t n;
  int32_t d;
  int32_t k;
  float *C_inout;   /* k x d: initial centres in, final centres out          */
  int32_t *labels;  /* n: final assignment                                   */
  float *mindist;   /* n, nullable: squared distance to the assigned centre */
  double *sse_hist; /* max_iter+1, nullable: SSE of every assignment pass   */
  int32_t max_iter; /* t_max                                                 */
  double tol;       /* tau: stop when the largest centre move is < tol       */
  km_stats *stats;  /* HOST pointer, nullable: filled on completion          */
} km_problem;

/* ---- context ---------------------------------------------------------------
 * Creates a context bound to HIP device `device`: it owns the library's
 * device workspace (grown on demand) and the tile-shape cache.  Returns
 * KM_ERR_DEVICE if the device is not a gfx950 GPU. */
int32_t kmeans_context_create(int32_t device, km_context **out);
int32_t kmeans_context_destroy(km_context *ctx);

/* ---- one assignment pass ----------------------------------------------------
 * For every point x_i and centre c_j computes the mixed-precision squared
 * distance of Algorithm alg:mp-dist (expanded formula on quantised inputs,
 * reliability test, FP64 direct correction of flagged pairs, result in FP32)
 * and assigns x_i to the centre with the smallest value (first index among
 * equal values of the expanded-formula term; Algorithm alg:mp-kmeans).
 * Outputs:
 *   labels  [n] int32
 *   mindist [n] FP32, nullable: ||x_i - c_{label_i}||^2 recomputed in FP64 by
 *           the direct formula from the FP32 data and rounded once to FP32
 *   sse     [1] FP64 device scalar, nullable: sum of those FP64 distances
 *   stats   host, nullable (forces a wait): counts, alpha, data status
 * With KM_LABELS_HINT in flags, labels is also read: entries in [0,k) seed
 * each point's running best (others are ignored); the outputs are identical
 * to a call without the flag, the sweep only skips saving blocks that cannot
 * hold the winner.  kmeans_lloyd and the batched solves seed every round
 * after the first from the previous round's labels.
 * Limits: 1 <= d <= 256, 1 <= k <= 65536, 1 <= n.  k > n is allowed. */
int32_t kmeans_assign(km_context *ctx, const float *X, int64_t n, int32_t d,
                      const float *C, int32_t k, const km_precision *prec,
                      int32_t *labels, float *mindist, double *sse,
                      km_stats *stats, void *stream, uint32_t flags);

/* ---- one assignment pass with its per-pair fallback decisions --------------
 * The pass of kmeans_assign (same labels, same counters), recording which
 * pairs the reliability test eq:quantis-reliability-test sent to the
 * high-precision fallback of eq:fallback-rule-mp (Algorithm alg:mp-dist):
 * flagged [n*k] uint8, device, row-major by point, owned by the caller; the
 * library clears it and writes 1 for every flagged pair, so that the count
 * of ones equals stats->n_corrected.  A pass whose threshold flags every
 * pair (alpha >= 2.5, run by the direct kernel) fills it with ones; the
 * plain FP64 pass and a pass without a test leave it zero.  For diagnostics
 * and tests: it shows where the expanded formula cancels.  mindist and the
 * SSE are not produced (stats->sse_last is the refined SSE when stats is
 * given).  Errors as kmeans_assign, KM_ERR_ARG for a NULL flagged. */
int32_t kmeans_assign_flags(km_context *ctx, const float *X, int64_t n,
                            int32_t d, const float *C, int32_t k,
                            const km_precision *prec, int32_t *labels,
                            uint8_t *flagged, km_stats *stats, void *stream,
                            uint32_t flags);

/* ---- one assignment pass without any allocation -----------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * pass, arguments, outputs and results as kmeans_assign (bitwise), but the
 * pass's workspace (quantised centres, per-centre constants, per-workgroup
 * partials, status word and result record) lives in a fixed device array of
 * KM_STATIC_SCRATCH_BYTES that the library holds on each device for the life
 * of the process; the call makes no device allocation (descriptors go
 * through the context's pinned upload ring, allocated when the context was
 * created).  A pass whose workspace would exceed the array returns
 * KM_ERR_UNSUPPORTED before enqueueing anything (roughly k*d <= 2^21 and
 * n <= 2^24 fit).  Every call on a device shares that device's array and
 * keeps the last call's contents: calls that overlap on one device (other
 * streams, other contexts, other host threads) race and must be ordered by
 * the caller.  Kernel timing (kmeans_timing_enable) is not recorded. */
#define KM_STATIC_SCRATCH_BYTES (24u << 20)
int32_t kmeans_assign_static(km_context *ctx, const float *X, int64_t n,
                             int32_t d, const float *C, int32_t k,
                             const km_precision *prec, int32_t *labels,
                             float *mindist, double *sse, km_stats *stats,
                             void *stream, uint32_t flags);

/* ---- one centre update (eq:center, Algorithm alg:mp-kmeans) -----------------
 * C_new[j] = fl32( (sum_{i: labels_i = j} x_i) / m_j ) with the sums taken in
 * FP64 in a fixed order that does not depend on the launch (points of a
 * cluster in ascending index, in chunks of 64); an empty cluster keeps
 * C_old[j].  counts [k] int64 and shift [1] FP64 (max_j ||C_new-C_old||) are
 * device outputs, nullable.  sse [1] FP64 device scalar, nullable: the SSE of
 * the given labels against C_old (eq:sse), sum_i ||x_i - C_old[label_i]||^2
 * in FP64 from the FP32 data, accumulated in a fixed order while the update
 * reads every point's row -- the SSE of the assignment pass that produced
 * the labels, without that pass refining its winners.  labels must lie in
 * [0,k). */
int32_t kmeans_update(km_context *ctx, const float *X, int64_t n, int32_t d,
                      const int32_t *labels, int32_t k, const float *C_old,
                      float *C_new, int64_t *counts, double *shift, double *sse,
                      void *stream, uint32_t flags);

/* ---- Lloyd's algorithm (Algorithm alg:mp-kmeans) ---------------------------
 * C_inout holds the initial centres on entry and the final ones on exit.
 * Runs up to max_iter rounds of (assignment pass, centre update), stopping
 * after a round whose largest centre move is < tol (tol <= 0: never; a
 * positive tol costs one device-to-host read per round, or one per call when
 * the rounds run in one launch), then one final assignment pass whose result
 * fills labels / mindist.  sse_hist (device, nullable, max_iter+1 entries)
 * receives the SSE of each assignment pass in order, the final one last.
 * max_iter = 0 performs the final pass only.
 * With KM_ROUND_LAUNCH in flags, small problems (FP16/BF16 operands,
 * d <= 32, k <= 64) run all their rounds in one persistent launch: a grid of
 * co-resident workgroups that assigns, updates and tests for convergence on
 * the device, with grid-wide waits between the phases, so a positive tol
 * costs no read per round and the host issues one launch per solve.  The
 * results are bitwise those of one launch per phase (the default, which is
 * the faster of the two when tol <= 0).  KM_ERR_DEVICE if such a wait ever
 * gives up (it never should; the launch then ends instead of hanging; the
 * KM_ROUND_SPIN_LIMIT environment variable caps a wait's polls, for tests
 * of that path).
 * Normalisation of the data (first line of the algorithm) is the caller's. */
int32_t kmeans_lloyd(km_context *ctx, const float *X, int64_t n, int32_t d,
                     int32_t k, float *C_inout, int32_t max_iter, double tol,
                     const km_precision *prec, int32_t *labels, float *mindist,
                     double *sse_hist, km_stats *stats, void *stream,
                     uint32_t flags);

/* ---- Lloyd's algorithm with a precision schedule ---------------------------
 * The precision guidance of Section 6 (closing implications paragraph):
 * while centre-point distances are large, uniform low precision suffices;
 * near convergence, cancellation calls for the fallback.  The paper gives no
 * switching criterion; this entry point uses one the host loop can check
 * each round: rounds use `early` while the round's SSE falls by at least the
 * fraction switch_rel of the previous round's SSE, for at most max_early
 * rounds; every later round and the final pass use `late`.  With
 * max_early = 0 it is kmeans_lloyd with `late`.  Each early round costs one
 * device-to-host read (the round's SSE and shift).  *switch_round (host,
 * nullable) receives the index of the first round in `late` (the number of
 * rounds if the final pass is the first).  stats sums the corrected pairs of
 * both phases; sse_last is the final pass's.  Other arguments as
 * kmeans_lloyd. */
int32_t kmeans_lloyd_schedule(km_context *ctx, const float *X, int64_t n,
                              int32_t d, int32_t k, float *C_inout,
                              int32_t max_iter, double tol,
                              const km_precision *early,
                              const km_precision *late, double switch_rel,
                              int32_t max_early, int32_t *labels,
                              float *mindist, double *sse_hist,
                              km_stats *stats, int32_t *switch_round,
                              void *stream, uint32_t flags);

/* ---- k-means++ seeding (D^2 weighting) ---------------------------------------
 * The seeding the paper's introduction names as combinable with the method
 * (Arthur and Vassilvitskii).  C_out (device, k x d) receives k rows of X:
 * row 0 is point floor(u_0 n); row i >= 1 is the first point p whose running
 * sum of weights w, in point order, exceeds u_i * sum(w), where w_p is the
 * smallest ||x_p - c||^2 over the rows chosen so far (FP64, coordinates in
 * index order).  The FP64 sums run in a fixed order (per 1024-point block,
 * then blocks, then the chosen block's points), so the rows depend only on X
 * and the uniforms.  uniforms: host array of k values in [0, 1) (the random
 * draws are the caller's).  idx_out (device, k int32, nullable) receives the
 * chosen point indices.  If every weight is zero (all points coincide with
 * chosen rows) row i is point floor(u_i n).  1 <= k <= min(n, 65536),
 * d <= 1024; 2k - 1 launches, one FP64 read of X per row. */
int32_t kmeans_seed_pp(km_context *ctx, const float *X, int64_t n, int32_t d,
                       int32_t k, const double *uniforms, float *C_out,
                       int32_t *idx_out, void *stream, uint32_t flags);

/* ---- clustering agreement (host arrays; no device work) ----------------------
 * The measures the paper reports next to the SSE (Section 6): labels_a and
 * labels_b are n int32 labels (any values) of the same points.
 * kmeans_ari: adjusted Rand index (pair counting, chance-corrected).
 * kmeans_ami: adjusted mutual information (Vinh, Epps and Bailey), natural
 *   logarithm, the arithmetic mean of the two entropies as normaliser, the
 *   expected mutual information under fixed margins.
 *   Both are 1.0 when both labelings put every point in one cluster or every
 *   point in its own.
 * kmeans_label_diff: the segmentation Diff of Section 6.3, the fraction of
 *   points whose labels differ after the one-to-one matching of cluster ids
 *   that agrees on the most points (KM_ERR_UNSUPPORTED above 4096 ids).
 * Each returns KM_OK or KM_ERR_ARG (NULL pointer, n < 1). */
int32_t kmeans_ari(const int32_t *labels_a, const int32_t *labels_b, int64_t n,
                   double *ari);
int32_t kmeans_ami(const int32_t *labels_a, const int32_t *labels_b, int64_t n,
                   double *ami);
int32_t kmeans_label_diff(const int32_t *labels_a, const int32_t *labels_b,
                          int64_t n, double *diff);

/* ---- many independent problems in one set of launches ----------------------
 * Solves count problems (device pointers) with the same precision.  Each
 * phase of a Lloyd round is one launch over a work list that spans all
 * problems, so small problems share the GPU.  Every problem's arithmetic is
 * identical to a kmeans_lloyd call on it alone (bitwise).  Per-problem tol
 * stopping is honoured at round granularity.  With KM_ROUND_LAUNCH in flags
 * the problems that kmeans_lloyd's persistent launch serves run all their
 * remaining rounds (after any sweep-length tuning rounds) in one persistent
 * launch per kernel shape, each with its own max_iter and tol; results are
 * bitwise the same. */
int32_t kmeans_solve_batch(km_context *ctx, km_problem *probs, int32_t count,
                           const km_precision *prec, void *stream,
                           uint32_t flags);

/* ---- materialised distances (reports and tests; not on the hot path) -------
 * D [m x k] FP32: the per-pair value the assignment pass uses (the
 * expanded-formula value of kept pairs, the FP64 direct value rounded to FP32
 * for corrected pairs); flagged [m x k] uint8, nullable: 1 where the pair was
 * corrected.  Same kernels and arithmetic as kmeans_assign. */
int32_t kmeans_pairwise(km_context *ctx, const float *X, int64_t m, int32_t d,
                        const float *C, int32_t k, const km_precision *prec,
                        float *D, uint8_t *flagged, void *stream,
                        uint32_t flags);

/* ---- quantisation (tests) ---------------------------------------------------
 * out[i] = bits of the low-precision value of in[i] (round to nearest even,
 * gradual underflow, overflow to infinity) as used by every kernel; low is
 * KM_LOW_FP16 or KM_LOW_BF16. */
int32_t kmeans_quantize(km_context *ctx, const float *in, int64_t count,
                        int32_t low, uint16_t *out, void *stream,
                        uint32_t flags);

/* The threshold alpha the library applies for (prec, d); -1 when the mode
 * has no fallback and +inf when every pair is corrected.  Host only. */
int32_t kmeans_alpha(const km_precision *prec, int32_t d, double *alpha_out);

/* ---- serving: continuous batching -------------------------------------------
 * A server owns a device arena of at most hbm_budget_bytes and a scheduler
 * thread.  kmeans_submit copies nothing yet: the request waits until its
 * device footprint fits the budget and fewer than max_active requests run,
 * then its data are copied in and it joins the running set at the next round
 * boundary.  Every round performs one Lloyd round for all running requests
 * with batched launches; finished requests are copied back to their host
 * buffers and leave.  A request's results do not depend on what else runs.
 * A request whose footprint exceeds the whole budget fails with
 * KM_ERR_OOM; malformed requests fail with their own error code. */
int32_t kmeans_server_create(km_context *ctx, size_t hbm_budget_bytes,
                             int32_t max_active, km_server **out);
int32_t kmeans_submit(km_server *srv, const km_problem *host_req,
                      const km_precision *prec, uint64_t *ticket);
/* KM_OK when done (host buffers filled), KM_PENDING after timeout_ms
 * (0 = do not wait, < 0 = wait forever), or the request's error code.  A
 * finished ticket stays queryable until kmeans_server_destroy. */
int32_t kmeans_poll(km_server *srv, uint64_t ticket, int32_t timeout_ms);
int32_t kmeans_cancel(km_server *srv, uint64_t ticket);
/* Waits for the scheduler to finish running requests, cancels queued ones
 * and frees the arena. */
int32_t kmeans_server_destroy(km_server *srv);

/* ---- kernel timing (benchmarks) ----------------------------------------------
 * While enabled, every launch of the assignment kernel (the fused
 * mixed-precision kernel or the FP64 direct kernel) and every persistent
 * round launch of kmeans_lloyd (all its rounds: one entry) is bracketed by
 * two HIP events recorded on the launch's stream.  kmeans_timing_enable resets the
 * record.  kmeans_timing_read waits for the recorded events and copies up to
 * `max` durations (milliseconds, launch order) into ms_out; *count receives
 * the number recorded. */
int32_t kmeans_timing_enable(km_context *ctx, int32_t enable);
int32_t kmeans_timing_read(km_context *ctx, float *ms_out, int32_t max,
                           int32_t *count);

/* ---- tuning cache ---------------------------------------------------------
 * kmeans_solve_batch times the first rounds of its small-problem launches
 * with 2, 4, 8, 16 and 32 groups of 32 points per wave and keeps the
 * fastest; the choice is remembered per shape bucket (low format,
 * correction precision, threshold on/off, largest kernel row capacity,
 * largest padded k, total points rounded down to a power of two) in the
 * context, and a later batch of the same bucket uses it without timing.
 * Results never depend on the choice.
 * kmeans_tune_cache: a file that makes the choices persistent (read now if it
 *   exists, rewritten after every new choice; one text line per bucket: key,
 *   groups per wave, the five times in ms).  NULL or "" keeps them in
 *   memory only.  Returns KM_OK or KM_ERR_ARG.
 * kmeans_tune_dump: the cache as that text, NUL-terminated and cut to cap-1
 *   bytes; returns the full length (call with cap 0 to size the buffer). */
int32_t kmeans_tune_cache(km_context *ctx, const char *path);
int64_t kmeans_tune_dump(km_context *ctx, char *buf, int64_t cap);

/* Human-readable text for a status code (static storage). */
const char *kmeans_status_string(int32_t status);

#ifdef __cplusplus
}
#endif
#endif /* KMEANS_MI355X_H */
