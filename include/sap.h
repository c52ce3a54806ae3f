/*
 * sap.h -- C ABI of the MI355X (gfx950) Secant-Avoidance Projection library.
 *
 * The method (Kvinge, Farnell, Kirby, Peterson, "A GPU-Oriented Algorithm
 * Design for Secant-Based Dimensionality Reduction", 2018, Sec. 4 and
 * Algorithm 1) looks for an n x k projection P with orthonormal columns that
 * maximises the smallest projected unit-secant norm
 *         r_ij = || P^T (x_i - x_j) || / || x_i - x_j ||     (i < j)
 * over a point cloud X (N x n).  One iteration evaluates every r_ij, reduces
 * to the global minimum and its pair, and rotates span(P) toward that worst
 * secant (argmax basis vector, modified Gram-Schmidt, alpha shift).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers on the handle's device unless
 *    stated otherwise; result structs are HOST memory.
 *  - X is N x n row-major with leading dimension ldx >= n (elements), FP64
 *    or FP32.  X is BORROWED: the caller keeps it alive and unchanged until
 *    sap_destroy.  Every other buffer is owned by the library.
 *  - P arguments are n x k row-major, contiguous (element (l, c) at l*k + c).
 *  - Pairs are unordered, i < j, indexed q = i*N - i*(i+1)/2 + (j - i - 1).
 *    Argmin ties are broken by the smallest (i, j).
 *  - Work is enqueued on the stream given to sap_init (or sap_set_stream).
 *    Only sap_init, sap_min_secant, sap_step with a non-NULL result, sap_set_P,
 *    sap_info, sap_softmin_bwd and sap_profile_read synchronise that stream.
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - Errors are returned as status codes, never thrown.  SAP_ERR_DEVICE
 *    poisons the handle: afterwards only sap_last_error and sap_destroy work.
 *
 * Two forms of the per-iteration pass are provided:
 *  - SAP_PLAIN stores every unit secant once (n x p, component-major, the
 *    paper's "secants as columns of S", Sec. 4) in the dtype of X and streams
 *    it from HBM each iteration;
 *  - SAP_FUSED never stores a secant: it forms Y = (X - mean) P on the
 *    matrix cores in FP64, rounds Y to FP32, and scores (i, j) tiles as
 *    ||y_i - y_j||^2 * (1/d_ij^2) with the denominators precomputed once.
 * Both forms rescore, in FP64 from X, every pair whose coarse value lies in a
 * window proven (from the rounding-error bound of the coarse pass) to
 * contain the true minimum, so the reported minimum and pair are those of
 * an FP64 evaluation.  The fused form keeps pairs shorter than a cutoff D_c
 * out of the coarse pass, because there the coarse error, which grows like
 * 1/d, would swamp them: with the FP64 GEMM it bounds them from the unrounded
 * FP64 Y and evaluates exactly from X only those that may hold one of their
 * block's two smallest values; otherwise it evaluates them all exactly.
 */
#ifndef SAP_H
#define SAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sap_ctx *sap_handle;

typedef enum {
    SAP_OK = 0,
    SAP_ERR_INVALID_ARG = 1,      /* bad size, range, pointer or combination      */
    SAP_ERR_NONFINITE = 2,        /* NaN or Inf in X or P                          */
    SAP_ERR_NO_PAIRS = 3,         /* every pair is a duplicate or shorter than l   */
    SAP_ERR_OUT_OF_MEMORY = 4,    /* device allocation failed                      */
    SAP_ERR_DEVICE = 5,           /* HIP runtime error; the handle is poisoned     */
    SAP_ERR_NOT_ORTHONORMAL = 6,  /* max |P^T P - I| > 1e-6                        */
    SAP_ERR_POISONED = 7,         /* handle unusable after an earlier device error */
    SAP_ERR_UNSUPPORTED = 8,      /* valid request outside this build's limits     */
    SAP_ERR_CAPACITY = 9          /* a library-owned list would exceed its cap     */
} sap_status;

enum { SAP_F64 = 0, SAP_F32 = 1 };                       /* dtype of X           */
enum { SAP_PLAIN = 0, SAP_FUSED = 1 };                   /* form of the pass     */
enum { SAP_STEP_LITERAL = 0, SAP_STEP_NORMALIZED = 1 };  /* reading of the shift */
/* Arithmetic of the fused form's Y = (X - mean) P (the projected points the
 * coarse pass differences): FP64 on the matrix cores (default; the coarse
 * error bound is then that of rounding Y to FP32), FP32 or BF16 inputs with
 * FP32 accumulation (cheaper operands, a proportionally wider rescoring
 * window; see sap_info's e_abs). */
enum { SAP_GEMM_F64 = 0, SAP_GEMM_F32 = 1, SAP_GEMM_BF16 = 2 };

/* Configuration: Algorithm 1's inputs (target dimension k, shift alpha), the
 * length threshold l of Sec. 7 (min_len), and how the evaluation is carried
 * out.
 *   N >= 2, 1 <= k <= min(n, 16), n*(k+3) <= 19200 (the FP64 update keeps its
 *   vectors in LDS), alpha in [0, 1], min_len >= 0.
 *   rule: SAP_STEP_LITERAL combines the unnormalised P P^T s and s - P P^T s
 *         (the wording of Sec. 4 and Algorithm 1); SAP_STEP_NORMALIZED
 *         combines their unit vectors.
 *   close_d: fused form only; pairs with d < close_d are evaluated in FP64
 *         every iteration.  < 0 selects it automatically: the cutoff at
 *         which the coarse error bound e_abs (see sap_info) is about 4e-6.
 *         close_cap bounds that list (0 = min(2^20, max(1024, p / n)));
 *         an automatic cutoff is lowered until the list fits, an explicit one
 *         that does not fit fails with SAP_ERR_CAPACITY.
 *   cand_cap: capacity of each wavefront's list of rescoring candidates,
 *         1..128 (0 = 128).  A list that fills up keeps its smallest coarse
 *         values; if that drops a pair of the proven window the result is
 *         reported with certified = 0 (it is then the best of the pairs that
 *         were rescored).
 *   gemm: SAP_GEMM_F64 | SAP_GEMM_F32 | SAP_GEMM_BF16 (fused form). */
typedef struct {
    int64_t N;
    int32_t n, k;
    int32_t dtype;      /* SAP_F64 | SAP_F32                        */
    int32_t form;       /* SAP_PLAIN | SAP_FUSED                    */
    int32_t rule;       /* SAP_STEP_LITERAL | SAP_STEP_NORMALIZED   */
    int32_t close_cap;
    int32_t cand_cap;
    int32_t gemm;       /* SAP_GEMM_F64 | SAP_GEMM_F32 | SAP_GEMM_BF16 */
    double alpha;
    double min_len;
    double close_d;
} sap_config;

/* One evaluation of the secant set (Algorithm 1, the argmin step: the worst
 * secant of the current P and its projected norm). */
typedef struct {
    double min_norm;     /* FP64 min of ||P^T s|| over kept pairs              */
    double runner_up;    /* a lower bound of the second-smallest ||P^T s||
                            (lexicographic order), exact if runner_up_exact   */
    int64_t i, j;        /* the pair of min_norm (i < j), smallest (i, j) on ties */
    int64_t pair_index;  /* q(i, j)                                            */
    double coarse_min;   /* smallest coarse (FP32/FP64-pass) value; -1 if none */
    double window;       /* coarse values within this of coarse_min were rescored */
    int32_t certified;   /* 1: the pair is provably the FP64 argmin            */
    int32_t runner_up_exact;
    int32_t n_rescored;  /* pairs evaluated in FP64 this iteration             */
    int32_t t;           /* basis vector replaced by the update (0-based)      */
    int32_t n_units;     /* work items of the pass that held candidates        */
    int32_t reserved;
} sap_min_result;

/* Sizes and precision parameters of a handle (host struct). */
typedef struct {
    int64_t n_pairs;        /* kept pairs |Pi|                                  */
    int64_t n_dropped;      /* duplicates + pairs shorter than min_len          */
    int64_t n_close;        /* fused: pairs evaluated in FP64 every iteration    */
    double close_d;         /* fused: cutoff D_c actually used                   */
    double e_abs, e_rel;    /* coarse error bound |r~ - r| <= e_abs + e_rel r    */
    double radius;          /* max_i ||x_i - mean||                             */
    int64_t bytes_per_iter; /* algorithmic HBM bytes of one pair pass            */
    int64_t device_bytes;   /* device memory owned by the handle                */
    int64_t n_tiles;        /* tiles (fused) or chunks (plain) of the pair pass  */
} sap_info_t;

/* Create a handle for Algorithm 1's inputs (Sec. 4: the secant set of X --
 * every unit secant (x_i - x_j)/||x_i - x_j||, i < j, minus those shorter than
 * min_len, Sec. 7 -- the target dimension and the shift) and the starting
 * projection P0 (n x k FP64, orthonormal columns).  Validates, allocates,
 * checks that X is finite and P0 orthonormal, and precomputes the secant
 * array (plain form: the matrix S with the secants as columns, Sec. 4) or the
 * tile-packed 1/d^2 array and the short-pair list (fused form).  stream is a
 * hipStream_t (NULL = the null stream).  Errors: SAP_ERR_INVALID_ARG,
 * SAP_ERR_UNSUPPORTED, SAP_ERR_NONFINITE, SAP_ERR_NOT_ORTHONORMAL,
 * SAP_ERR_NO_PAIRS, SAP_ERR_CAPACITY, SAP_ERR_OUT_OF_MEMORY, SAP_ERR_DEVICE.
 * On failure *out is NULL. */
sap_status sap_init(const sap_config *cfg, const void *X, int64_t ldx,
                    const double *P0, void *stream, sap_handle *out);

/* Algorithm 1's argmin step for the current P (Sec. 4: the column of P^T S
 * of smallest norm): min, argmin, runner-up and the rescoring record.
 * Synchronises. */
sap_status sap_min_secant(sap_handle h, sap_min_result *out);

/* One iteration of Algorithm 1 (Sec. 4): the argmin step, then the update of
 * P from the worst secant s -- t = argmax_c |<p_c, s>| (smallest c on ties;
 * if every product is zero, p_1 is replaced by s), modified Gram-Schmidt on
 * (P P^T s, the other basis vectors in order), and the first vector set to the
 * unit vector along (1 - alpha) P P^T s + alpha (s - P P^T s) -- in FP64.
 * For k <= 12 (k <= 8 when n <= 64) the Gram-Schmidt step is carried out on
 * the vectors' coordinates in the basis P, whose inner products equal the
 * vectors' own for orthonormal P; the new vectors are P times them.
 * With out == NULL it is fully asynchronous; otherwise it synchronises and
 * reports the evaluation that drove the update. */
sap_status sap_step(sap_handle h, sap_min_result *out_or_null);

/* Algorithm 1 from the current P: iters updates and iters+1 evaluations (the
 * last one scores the returned P).  Traces are device buffers of iters+1
 * entries: min (FP64), (i, j) as 2 int64 per entry, certified (int32).
 * ij_trace and cert_trace may be NULL.  Asynchronous.  The fused form runs
 * each iteration's selection and update in the same launch as the next
 * iteration's Y GEMM (two launches per iteration); results are those of
 * iters calls of sap_step followed by sap_min_secant. */
sap_status sap_run(sap_handle h, int32_t iters, double *min_trace,
                   int64_t *ij_trace, int32_t *cert_trace);

/* The current projection P of Algorithm 1 (Sec. 4: n x k, orthonormal
 * columns p_1..p_k): copy the FP64 master out (n x k row-major device buffer;
 * asynchronous) / replace it.  sap_set_P checks orthonormality
 * (max |P^T P - I| <= 1e-6, else SAP_ERR_NOT_ORTHONORMAL; NaN/Inf:
 * SAP_ERR_NONFINITE) and synchronises. */
sap_status sap_get_P(sap_handle h, double *P_out);
sap_status sap_set_P(sap_handle h, const double *P);

/* Algorithm 1's initial projection (Sec. 4; Algorithm 1, step 2): P(1) =
 * the first k columns of U, where S = U Sigma V^T is the SVD of the secant
 * matrix S (the handle's kept unit secants as columns) -- the top-k
 * eigenvectors of S S^T = sum_{kept i<j} s_ij s_ij^T.  Computed on the device
 * in FP64 without forming S: S S^T = sum_i (x_i - mean) z_i^T with
 * z_i = sum_j (x_i - x_j) / d_ij^2 (direct differences), then a subspace
 * iteration with Rayleigh-Ritz until the largest residual
 * ||S S^T p_c - sigma_c^2 p_c|| / sigma_1^2 of the k vectors is <= 1e-12 (at
 * most 400 rounds).  Each column is signed so that its largest-magnitude
 * component is positive (the first such component on ties).  Writes P
 * (n x k row-major device buffer; may be NULL) and info (host; may be
 * NULL); with set_P != 0 the result also becomes the handle's current P.
 * Device scratch of about 4 N^2 + 8 N n + 16 n^2 bytes is allocated and
 * freed by the call, which synchronises.  Errors: SAP_ERR_INVALID_ARG,
 * SAP_ERR_OUT_OF_MEMORY, SAP_ERR_DEVICE. */
typedef struct {
    double sigma[16];     /* the k largest singular values of S, descending; 0 beyond k */
    double residual;      /* max over the k vectors of the relative residual above     */
    double ms;            /* device time of the whole computation                     */
    int32_t iters;        /* rounds of the subspace iteration                         */
    int32_t converged;    /* 1 when residual <= 1e-12                                 */
} sap_pca_info;

sap_status sap_pca_init(sap_handle h, double *P_out, sap_pca_info *info, int32_t set_P);

/* Change the stream later work is enqueued on (no device work). */
sap_status sap_set_stream(sap_handle h, void *stream);

/* Sizes of the secant set (Sec. 4, Sec. 7) and the error-bound parameters of
 * the coarse evaluation.  Synchronises. */
sap_status sap_info(sap_handle h, sap_info_t *out);

/* Soft-min surrogate of the minimum (not in the paper; a differentiable
 * stand-in for Algorithm 1's min; fused form only):
 *   L = -tau log sum_{kept i<j} exp(-r_ij / tau),   r_ij = ||P^T s_ij||,
 * for the FP32 projection P (n x k row-major device buffer; it need not be
 * orthonormal).  r_ij is the coarse FP32 value of the fused pass (its error
 * bound is that of sap_info), or FP64 for the short pairs.  L is written to
 * loss[0] (device FP32).  The handle keeps what the backward needs (its own
 * FP64 copy of P, Y and L), so sap_softmin_bwd differentiates at the P of the
 * latest sap_softmin_fwd, and must be called with that forward's tau (else
 * SAP_ERR_INVALID_ARG); a later forward replaces the saved state.
 * tau in [1e-6, 1e6].  SAP_PLAIN handles return SAP_ERR_UNSUPPORTED.
 * Asynchronous. */
sap_status sap_softmin_fwd(sap_handle h, const float *P, double tau,
                           float *loss);

/* Gradient of the soft-min at the P of the latest forward:
 *   dP = g dL/dP = g sum_{kept i<j} w_ij s_ij (P^T s_ij)^T / r_ij,
 * w_ij = exp(-(r_ij - L)/tau) (sum w = 1), g = grad_loss[0] (device FP32).
 * Contracted as (X - mean)^T Z with z_i = sum_j a_ij (y_i - y_j),
 * a_ij = w_ij / (d_ij^2 r_ij): the weights are recomputed from Y and 1/d^2,
 * never stored.  Pairs with r_ij = 0 contribute nothing.  dP is n x k
 * row-major FP32, overwritten.  Deterministic.  P must hold, bit for bit,
 * the projection passed to that forward, and tau must be the forward's:
 * otherwise SAP_ERR_INVALID_ARG (P is compared with the forward's copy, so
 * this call synchronises the stream before enqueuing the backward). */
sap_status sap_softmin_bwd(sap_handle h, const float *P, double tau,
                           const float *grad_loss, float *dP);

/* Per-kernel timing of the iteration, for roofline reporting.  While enabled,
 * every kernel launched by sap_min_secant / sap_step / sap_run (and by
 * sap_softmin_fwd / sap_softmin_bwd) is timed by the start and end
 * timestamps of its own dispatch (hipExtLaunchKernelGGL events on the
 * handle's stream; the work itself is unchanged).  sap_profile_read
 * synchronises, returns the summed durations and launch counts since the
 * last read, and restarts the accumulation.
 * Slots: 0 = Y GEMM (fused form), 1 = pair pass (with the window pairs'
 * FP64 rescoring and the fused form's FP64 short pairs), 2 = selection:
 * record and update; soft-min:
 * 3 = forward tile pass, 4 = backward tile pass, 5 = the other soft-min
 * launches (P load, Y GEMM, short pairs, merges, the (X - mean)^T Z
 * contraction); 6 = sap_run in the fused form: selection, record and
 * update fused with the next iteration's Y GEMM (slot 0 then counts the
 * run's first GEMM only); 7 is unused. */
typedef struct {
    double ms[8];
    int64_t launches[8];
} sap_profile_t;

sap_status sap_profile_enable(sap_handle h, int32_t on);
sap_status sap_profile_read(sap_handle h, sap_profile_t *out);

/* ------------------------------------------------------------------------
 * Batched SAP: many independent small problems in one launch.
 *
 * The paper runs Algorithm 1 on many small secant sets: once per target
 * dimension to read off the dimension of the data (Sec. 6.1, the sweep over
 * the projection dimension), on random subsamples of a set too large for its
 * secant matrix (Sec. 6.3, ten samples of 512 points), and with the length
 * threshold l of Sec. 7 to see through noise.  sap_batch_run runs B such
 * problems at once, each on its own workgroup, the whole run of iters
 * updates and iters+1 evaluations inside one kernel launch.
 *
 * A problem is Algorithm 1 on a point set S_s (rows of X listed by
 * set_points[set_offsets[s] .. set_offsets[s+1]), in that order; pairs and
 * their tie-break use these local indices) with its own k, alpha, rule and
 * start P0_b.  The set's threshold set_min_len[s] drops secants shorter than
 * l (Sec. 7) and duplicates.  Evaluation: Y = (X_S - mean) P in FP64 on the
 * matrix cores, coarse values ||y_i - y_j||^2 / d^2 rounded to FP32, and
 * FP64 rescoring from X of every pair in the proven window, as in the
 * single-problem handle (so there is no short-pair list); the update is the
 * handle's FP64 update.  Results are those of an FP64 evaluation whenever a
 * trace entry is certified.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t set;        /* its point set, 0 .. n_sets - 1                     */
    int32_t k;          /* target dimension, 1 .. min(n, 16)                  */
    int32_t rule;       /* SAP_STEP_LITERAL | SAP_STEP_NORMALIZED             */
    int32_t reserved;   /* 0                                                  */
    double alpha;       /* shift, in [0, 1]                                   */
} sap_batch_problem;

typedef struct {
    double init_ms;     /* device time of the per-set precomputation          */
    double run_ms;      /* device time of the run kernel (all problems)      */
    int64_t n_pairs;    /* kept pairs summed over the problems' sets          */
    int64_t scratch_bytes; /* device scratch the call used                    */
} sap_batch_stats;

/* Run the batch.  Host arrays: set_offsets (n_sets + 1, increasing, sets of
 * 2 .. 32768 points), set_points (set_offsets[n_sets] row indices into X,
 * each in [0, N)), set_min_len (n_sets, finite, >= 0; may be NULL = all 0),
 * problems (n_problems).  Device arrays: X (N x n, row-major, ldx >= n, FP64
 * or FP32, finite), P0 and P_out (problem b's n x k_b row-major block at
 * offset n * sum_{a<b} k_a doubles; every P0 block orthonormal to 1e-6),
 * min_trace (n_problems x (iters + 1) FP64: entry [b][it] is the minimum at
 * the it-th evaluation), ij_trace (n_problems x (iters + 1) x 2 int64, local
 * indices; may be NULL), cert_trace (n_problems x (iters + 1) int32; may be
 * NULL).  A set without any kept pair gives min = +inf, (-1, -1),
 * certified = 0, and P unchanged.  Limits: n * (k + 2) <= 16384 per problem
 * (the update's vectors live in LDS).  cand_cap as in sap_config (0 = 128).
 * stats may be NULL.  The call allocates its device scratch, synchronises
 * the stream, and frees the scratch before it returns.  Errors:
 * SAP_ERR_INVALID_ARG, SAP_ERR_NONFINITE, SAP_ERR_NOT_ORTHONORMAL,
 * SAP_ERR_UNSUPPORTED, SAP_ERR_OUT_OF_MEMORY, SAP_ERR_DEVICE; the message is
 * sap_last_error(NULL). */
sap_status sap_batch_run(const void *X, int32_t dtype, int64_t N, int32_t n, int64_t ldx,
                         int32_t n_sets, const int64_t *set_offsets, const int32_t *set_points,
                         const double *set_min_len, int32_t n_problems,
                         const sap_batch_problem *problems, const double *P0, int32_t iters,
                         int32_t cand_cap, double *P_out, double *min_trace, int64_t *ij_trace,
                         int32_t *cert_trace, void *stream, sap_batch_stats *stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as sap_batch_run -- same arguments, same kernels, same results --
 * except that its device scratch is a fixed array inside the library, 32 MiB
 * per GPU (each GPU the library runs on holds it until the process ends),
 * and that it creates no events (stats, if given, reports init_ms = run_ms =
 * -1).  It calls no hipMalloc or hipFree.  A batch that needs more scratch
 * than the array holds (stats->scratch_bytes of sap_batch_run tells) fails
 * with SAP_ERR_CAPACITY.  Every call on a GPU uses that GPU's one array and
 * leaves its contents behind (each call rewrites what it reads, and clears
 * its counters with a kernel): calls that overlap on one GPU (concurrent
 * streams or threads) race, and must be serialised by the caller. */
sap_status sap_batch_run_noalloc(const void *X, int32_t dtype, int64_t N, int32_t n, int64_t ldx,
                                 int32_t n_sets, const int64_t *set_offsets, const int32_t *set_points,
                                 const double *set_min_len, int32_t n_problems,
                                 const sap_batch_problem *problems, const double *P0, int32_t iters,
                                 int32_t cand_cap, double *P_out, double *min_trace, int64_t *ij_trace,
                                 int32_t *cert_trace, void *stream, sap_batch_stats *stats);

/* Free everything the handle owns.  NULL is accepted. */
sap_status sap_destroy(sap_handle h);

/* Last error message of the handle, or of the calling thread if h is NULL
 * (errors from sap_init).  Never NULL; valid until the next call on h. */
const char *sap_last_error(sap_handle h);

#ifdef __cplusplus
}
#endif

#endif /* SAP_H */
