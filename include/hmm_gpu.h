/*
 * hmm_gpu.h -- C ABI of the MI355X (gfx950) HMM inference library.
 *
 * The library evaluates, for many independent observation sequences at
 * once, the quantities of the paper's section 3 ("Algorithms"):
 *   - emission log-densities log b_j(y_t) (section 4 densities; 4.5 for the
 *     multivariate families),
 *   - the log-space forward recursion, eq. (loginit)/(logrec) of section 3.2,
 *     and the backward recursion computed "analogously" (section 3.2),
 *   - smoothed occupancies gamma_t(j) and pairwise occupancies xi_t(i,j)
 *     (definitions of section 3.1),
 *   - their gamma-weighted sufficient statistics pooled over all sequences
 *     (N_j and ybar_j of section 4, plus each family's sums), which is the
 *     E-step of Baum-Welch; multiple sequences are pooled (section 8 notes
 *     that the paper runs them one after another),
 *   - Viterbi decoding (section 3.3) and posterior decoding (section 3.4),
 *   - the weighted M-steps (section 4: closed forms 4.1, Gamma Newton 4.2,
 *     Student-t ECM 4.3, collapse guard 4.4, multivariate 4.5).
 *
 * Conventions shared by every call
 *   - All functions are extern "C" and return hmm_status.  A non-OK status
 *     leaves a message retrievable with hmm_last_error() (thread-local).
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary host memory.  The caller owns every buffer; the
 *     library allocates no device memory inside any call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued asynchronously; argument errors are detected on the
 *     host before anything is enqueued.  Results are valid once the stream
 *     has been synchronised.
 *   - Calls are reentrant when given distinct workspaces and outputs.
 *   - Numerical conditions found on the device are reported per sequence in
 *     seq_status (0 ok; 1 log-likelihood is -inf: no state path can emit
 *     the sequence; 2 a non-finite observation; 4 a model parameter is
 *     outside its domain, e.g. a variance <= 0).  Such sequences contribute
 *     nothing to pooled statistics.
 */
#ifndef HMM_GPU_H
#define HMM_GPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HMM_OK = 0,
    HMM_ERR_ARG = 1,            /* invalid argument (null pointer, bad size, T_b = 0, ...) */
    HMM_ERR_UNSUPPORTED = 2,    /* valid request this build does not implement */
    HMM_ERR_WORKSPACE = 3,      /* workspace missing or smaller than hmm_workspace_size */
    HMM_ERR_DEVICE = 4,         /* a HIP runtime call failed */
    HMM_ERR_PARAMS_UNSET = 5,   /* emission parameters (theta) not set */
    HMM_ERR_NUMERIC = 6         /* a parameter is outside its domain (variance <= 0, ...) */
} hmm_status;

/* Emission families.  theta is FP64, structure-of-arrays over the N states:
 *   HMM_GAUSSIAN       [mu(N), var(N)]                                   (4.1)
 *   HMM_GAMMA          [shape(N), rate(N)]  b(y) = rate^a y^(a-1) e^(-rate y) / Gamma(a), y > 0 (4.2)
 *   HMM_STUDENT_T      [mu(N), sigma(N), nu(N)] location-scale t         (4.3)
 *   HMM_POISSON        [lambda(N)]  y must be a non-negative integer value
 *   HMM_DIAG_GAUSSIAN  [mu(N*D), var(N*D)]  row j = state j              (4.5)
 *   HMM_FULL_GAUSSIAN  [mu(N*D), L(N*D*D)]  Sigma_j = L_j L_j^T, L_j lower
 *                       triangular, row-major                             (4.5)
 *   HMM_TABLE          no theta; `obs` holds log b_j(y_t) directly as
 *                       [sum T, N] (dim must equal N).  This covers any
 *                       family whose log-density the caller evaluates itself
 *                       (e.g. the discrete emissions of the paper's section 6.1). */
typedef enum {
    HMM_GAUSSIAN = 0,
    HMM_GAMMA = 1,
    HMM_STUDENT_T = 2,
    HMM_POISSON = 3,
    HMM_DIAG_GAUSSIAN = 4,
    HMM_FULL_GAUSSIAN = 5,
    HMM_TABLE = 6
} hmm_family;

/* Arithmetic of the recursions.
 *   HMM_PREC_F64 / HMM_PREC_F32: the batched path.  The log-space recursion
 *     is carried as a normalised vector (max entry in [1/2, 1)) plus an exact
 *     log offset (binary exponent sums and FP64 sums of per-step shifts), so
 *     lse_i[x_i + log a_ij] = c + log sum_i exp(x_i - c) a_ij with c = max x
 *     (the shift of section 3.2's lse).  Long sequences are cut into chunks
 *     whose transfer matrices are formed in parallel.
 *   HMM_PREC_PLAIN_F32 / HMM_PREC_PLAIN_F64: the paper's recursion taken
 *     literally on the GPU: one thread per sequence, N log-sum-exps of N terms
 *     per step, alpha and beta stored, separate kernels (the baseline).
 *   HMM_PREC_BF16_SCALED / HMM_PREC_F16_SCALED: the scaled (probability
 *     space) recursion that section 3.2 sets aside for its underflow, kept
 *     as a low-precision option for N > 64 and the multivariate families:
 *     the vector-matrix products run on the matrix cores with bf16 / fp16
 *     operands and FP32 accumulation, rescaled by a power of two at every
 *     step; alpha, gamma, the log offsets and the statistics stay FP32 / FP64.
 *     Their error against the FP64 path is a property of the format (about
 *     1e-5 relative on log P for fp16, 1e-4 .. 1e-3 for bf16 at N = 256). */
typedef enum {
    HMM_PREC_F64 = 0,
    HMM_PREC_F32 = 1,
    HMM_PREC_BF16_SCALED = 2,
    HMM_PREC_F16_SCALED = 3,
    HMM_PREC_PLAIN_F32 = 4,
    HMM_PREC_PLAIN_F64 = 5
} hmm_precision;

/* Operation selector for hmm_workspace_size. */
typedef enum {
    HMM_OP_EMISSION = 0,
    HMM_OP_FORWARD_BACKWARD = 1,
    HMM_OP_ESTEP = 2,
    HMM_OP_VITERBI = 3,
    HMM_OP_POSTERIOR_DECODE = 4
} hmm_op;

/* lambda = (pi, A, B) of section 3.1.  All pointers are device, FP64. */
typedef struct {
    int32_t n_states;       /* N >= 1 */
    int32_t dim;            /* D: 1 for the scalar families, N for HMM_TABLE */
    int32_t family;         /* hmm_family */
    int32_t reserved;       /* must be 0 */
    const double *log_pi;   /* [N] log initial probabilities (-inf allowed) */
    const double *log_A;    /* [N*N] log a_ij, row i = from state i, row-major (-inf allowed) */
    const double *theta;    /* family parameters (layout above); NULL -> HMM_ERR_PARAMS_UNSET */
} hmm_model;

/* A ragged batch of B sequences stored back to back.  Sequence b occupies
 * rows offsets[b] .. offsets[b+1]-1 of obs; every T_b must be >= 1. */
typedef struct {
    int64_t n_seq;              /* B >= 0 */
    const int64_t *offsets;     /* device [B+1], offsets[0] = 0 */
    const int64_t *h_offsets;   /* host [B+1], identical values (used for planning) */
    const void *obs;            /* device [sum T * D] row-major, float or double */
    int32_t obs_f64;            /* 1: obs is double; 0: obs is float */
    int32_t reserved;           /* must be 0 */
} hmm_batch;

/* Options of the emission M-steps (section 4).  hmm_mstep_default_opts
 * fills the paper's defaults. */
typedef struct {
    double eps_collapse;    /* N_j below this keeps theta_j (section 4.4); 1e-8 */
    double ridge;           /* full covariance gets + ridge * I (section 4.5); 1e-6 */
    double gamma_rtol;      /* Gamma shape Newton stops at |d a| <= rtol * a; 1e-12 */
    double nu_tol;          /* Student-t nu Newton stops at |d nu| < tol (section 4.3); 1e-6 */
    double nu_min, nu_max;  /* clamp of nu; 0.5 and 1e4 */
    int32_t max_iter;       /* Newton iteration cap; 100 */
    int32_t t_nu_printed;   /* 1: nu score exactly as printed in section 4.3 (without the
                               expected log-mixing term); 0 (default): corrected ECM score */
} hmm_mstep_opts;

/* Library version string (static storage). */
const char *hmm_version(void);

/* Message of the last non-OK status returned on this thread. */
const char *hmm_last_error(void);

/* Length of the pooled statistics vector of hmm_estep_stats, or 0 for an
 * invalid model.  Layout (FP64), with K the family block width:
 *   [0]                      sum_b log P(y^b | lambda) over sequences with status 0
 *   [1 .. N]                 sum_b gamma_1^b(i)
 *   [1+N .. 1+N+N*N)         sum_b sum_{t<T_b} xi_t^b(i,j), row-major (i, j)
 *   [1+N+N*N .. 1+2N+N*N)    N_j = sum_b sum_t gamma_t^b(j)
 *   [1+2N+N*N ..)            family block [N, K], per state j (d = y - current location):
 *     GAUSSIAN  K=2    sum g d, sum g d^2                       (d = y - mu_j)
 *     GAMMA     K=3    sum g y, sum g log y, sum g y^2
 *     STUDENT_T K=4    sum g u, sum g u d, sum g u d^2, sum g (log u - u),
 *                      u = (nu_j + 1) / (nu_j + d^2 / sigma_j^2)  eq. (utilde)
 *     POISSON   K=1    sum g y
 *     DIAG      K=2D   [sum g d_k], [sum g d_k^2]               (d = y - mu_j)
 *     FULL      K=D+D(D+1)/2  [sum g d_k], packed lower [sum g d_r d_c] (r >= c, row by row)
 *     TABLE     K=0 */
size_t hmm_stats_len(const hmm_model *model);

/* Bytes of workspace `op` needs for this model, batch and precision. */
hmm_status hmm_workspace_size(hmm_op op, const hmm_model *model, const hmm_batch *batch,
                              hmm_precision prec, size_t *bytes);

/* Emission log-densities log b_j(y_t) (the densities of section 4: 4.1
 * Gaussian and Poisson, 4.2 Gamma, 4.3 Student-t, 4.5 diagonal and full
 * covariance) for every step of every sequence.  log_b: device [sum T, N],
 * row-major, float for HMM_PREC_F32 / PLAIN_F32, double for F64 / PLAIN_F64
 * (the scaled precisions
 * write float).  Observations outside a family's support give -inf; non-finite
 * ones NaN.  ws: hmm_workspace_size(HMM_OP_EMISSION) bytes. */
hmm_status hmm_emission_logpdf(const hmm_model *model, const hmm_batch *batch,
                               hmm_precision prec, void *log_b, void *ws, size_t ws_bytes,
                               void *stream);

/* Forward-backward over the batch: the forward recursion of section 3.2
 * (eq. loginit / logrec, log-sum-exp as in that section), the backward
 * recursion it computes "analogously", and the smoothed occupancies
 * gamma_t(j) = P(q_t = j | y) of section 3.1.  loglik: device [B] FP64
 * log P(y^b | lambda) (-inf for status 1, NaN for status 2 and 4).
 * gamma: device [sum T, N] row-major, float or double as for
 * hmm_emission_logpdf, or NULL; rows of sequences with a non-zero status are
 * zero.  seq_status: device [B] int32 or NULL.
 * ws: hmm_workspace_size(HMM_OP_FORWARD_BACKWARD) bytes. */
hmm_status hmm_forward_backward(const hmm_model *model, const hmm_batch *batch,
                                hmm_precision prec, double *loglik, void *gamma,
                                int32_t *seq_status, void *ws, size_t ws_bytes, void *stream);

/* One Baum-Welch E-step: the forward-backward recursions of section 3.2,
 * the posteriors gamma and xi of section 3.1, and their weighted sums (the
 * N_j and family sums that the M-steps of section 4 read), pooled over the
 * sequences of the batch, into device `stats` (FP64, layout of
 * hmm_stats_len, overwritten).  loglik [B] and seq_status [B] are optional
 * device outputs.  The reduction order is fixed, so repeated calls on the
 * same inputs give bitwise-identical statistics.
 * ws: hmm_workspace_size(HMM_OP_ESTEP) bytes. */
hmm_status hmm_estep_stats(const hmm_model *model, const hmm_batch *batch, hmm_precision prec,
                           double *stats, double *loglik, int32_t *seq_status, void *ws,
                           size_t ws_bytes, void *stream);

/* Size of the static device area used by hmm_estep_stats_noalloc (64 MiB per
 * GPU, held from the library's load until the process ends). */
#define HMM_NOALLOC_SCRATCH_BYTES (64u << 20)

/* hmm_estep_stats for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments and results as hmm_estep_stats, but the workspace is a
 * static device array of HMM_NOALLOC_SCRATCH_BYTES in the library (one per
 * GPU, its address taken on the first call on each device).  No call
 * allocates or frees memory.  A batch whose hmm_workspace_size(HMM_OP_ESTEP)
 * exceeds the area is rejected with HMM_ERR_WORKSPACE before anything is
 * enqueued.  Every call on one GPU shares that GPU's area and leaves its
 * contents behind (each call initialises what it reads), so calls that may
 * overlap on one GPU (different streams or host threads) race: the caller
 * serialises them, e.g. on one stream. */
hmm_status hmm_estep_stats_noalloc(const hmm_model *model, const hmm_batch *batch,
                                   hmm_precision prec, double *stats, double *loglik,
                                   int32_t *seq_status, void *stream);

/* Viterbi decoding (section 3.3): the max-product recursion in log space
 * with backtrace.  path: device [sum T] int32 state indices (-1 on every
 * step of a sequence with no path or a non-finite observation); path_logp:
 * device [B] FP64 log-probability of the returned path (-inf if none, NaN
 * for a non-finite observation).  Ties are broken towards the lowest state
 * index.  n_ties: device [B] int32, or NULL: the near-ties met along the
 * returned path, i.e. decisions (the final state and each backpointer taken)
 * whose best and second-best scores, shifted per step, differ by less than
 * 1e-12; a path may differ from another exact evaluation only at such
 * decisions.  prec must be HMM_PREC_F64 or HMM_PREC_F32; N <= 64.
 * ws: hmm_workspace_size(HMM_OP_VITERBI) bytes. */
hmm_status hmm_viterbi(const hmm_model *model, const hmm_batch *batch, hmm_precision prec,
                       int32_t *path, double *path_logp, int32_t *n_ties, void *ws,
                       size_t ws_bytes, void *stream);

/* Posterior decoding (section 3.4): path[t] = lowest argmax_j gamma_t(j);
 * -1 on every step of a sequence whose status is not 0.  loglik: device [B]
 * FP64 or NULL.  ws: hmm_workspace_size(HMM_OP_POSTERIOR_DECODE) bytes. */
hmm_status hmm_posterior_decode(const hmm_model *model, const hmm_batch *batch,
                                hmm_precision prec, int32_t *path, double *loglik,
                                void *ws, size_t ws_bytes, void *stream);

/* Fill the section 4 defaults into *opts. */
void hmm_mstep_default_opts(hmm_mstep_opts *opts);

/* Transition M-step from pooled statistics (device, FP64):
 *   pi_i = sum_b gamma_1^b(i) / sum_i (...),  a_ij = Xi_ij / sum_j Xi_ij.
 * A row whose expected count sum_j Xi_ij is below opts->eps_collapse keeps
 * its values from model->log_A.  Outputs are device FP64 [N] and [N*N];
 * they may alias model->log_pi / model->log_A. */
hmm_status hmm_mstep_transitions(const hmm_model *model, const double *stats,
                                 const hmm_mstep_opts *opts, double *log_pi_out,
                                 double *log_A_out, void *stream);

/* Emission M-steps (section 4), one FP64 solve per state on the device, from
 * the pooled statistics of an E-step run with `model`'s current theta.
 * theta_out: device FP64, same layout as model->theta (may alias it).
 * collapsed: device int32 [N] or NULL: 0 updated, 1 N_j < eps_collapse
 * (parameters kept, section 4.4), 2 degenerate Gamma statistic (kept),
 * 3 covariance not positive definite (kept).  iters: device int32 [N] or
 * NULL: Newton iterations used (Gamma shape, Student-t nu).
 * Each function checks that model->family matches its name. */
hmm_status hmm_mstep_gaussian(const hmm_model *model, const double *stats,
                              const hmm_mstep_opts *opts, double *theta_out,
                              int32_t *collapsed, int32_t *iters, void *stream);
hmm_status hmm_mstep_gamma(const hmm_model *model, const double *stats,
                           const hmm_mstep_opts *opts, double *theta_out,
                           int32_t *collapsed, int32_t *iters, void *stream);
hmm_status hmm_mstep_student_t(const hmm_model *model, const double *stats,
                               const hmm_mstep_opts *opts, double *theta_out,
                               int32_t *collapsed, int32_t *iters, void *stream);
hmm_status hmm_mstep_poisson(const hmm_model *model, const double *stats,
                             const hmm_mstep_opts *opts, double *theta_out,
                             int32_t *collapsed, int32_t *iters, void *stream);
hmm_status hmm_mstep_diag_gaussian(const hmm_model *model, const double *stats,
                                   const hmm_mstep_opts *opts, double *theta_out,
                                   int32_t *collapsed, int32_t *iters, void *stream);
hmm_status hmm_mstep_full_gaussian(const hmm_model *model, const double *stats,
                                   const hmm_mstep_opts *opts, double *theta_out,
                                   int32_t *collapsed, int32_t *iters, void *stream);

/* Tuning: chunk length (time steps per chunk) of the batched path; 0 restores
 * the built-in choice.  Affects speed only, never the set of results beyond
 * rounding.  Returns HMM_ERR_ARG for values other than 0, 16, 32, 64.  When
 * nonzero it overrides the chunk length of the tuned variant. */
hmm_status hmm_set_chunk_len(int32_t steps);

/* Autotuning of the E-step's schedule.  Each batched route has a few
 * variants that compute the same quantities in a different schedule:
 *   N <= 8 (time-parallel chunks): variant 0/1/2 = chunks of 16/32/64 steps
 *     (FP64: 16/32);
 *   8 < N <= 64 and multivariate N <= 64 (FP64: N <= 32): variant 0/1/2/3 =
 *     forward and backward sweeps cut into segments of 1024 steps, whole
 *     sequences, 512 or 2048 steps (segments swept in parallel, each checked
 *     by a second sweep from its neighbour's vector and re-run in order where
 *     that finds no agreement);
 *   64 < N <= 256 (FP64: 32 < N <= 256) or multivariate N > 64: variant
 *     0/1/2 = the nominal, half or double number of row slices of the
 *     transition contraction;
 *   other routes: one variant.
 * hmm_autotune runs every variant of the route that (model, batch, prec)
 * takes, once to warm up and three times timed with hipEvents on `stream`
 * (it synchronises on them, so it is a set-up call, not for graph capture),
 * and keeps the fastest (median) for the call's key: device architecture,
 * family, N, D, precision, route and the batch's sequence count, mean and
 * longest length rounded up to powers of two.  Later calls with the same key
 * take that variant.  stats, loglik, seq_status, ws and ws_bytes are as for
 * hmm_estep_stats (ws: hmm_workspace_size(HMM_OP_ESTEP), which covers every
 * variant); they hold the last variant's results on return.  variant (host,
 * or NULL) receives the choice; ms (host float[4], or NULL) the median
 * milliseconds of each variant.  If the environment variable HMM_TUNE_CACHE
 * names a file, choices are appended to it ("key variant ms..." per line)
 * and read back at the first lookup of a later process. */
hmm_status hmm_autotune(const hmm_model *model, const hmm_batch *batch, hmm_precision prec,
                        double *stats, double *loglik, int32_t *seq_status, void *ws,
                        size_t ws_bytes, void *stream, int32_t *variant, float *ms);

/* Forces variant `variant` (clamped to the route's count) on every later call
 * of this process; -1 returns to tuned choices.  The environment variable
 * HMM_FORCE_VARIANT sets the initial value. */
hmm_status hmm_set_variant(int32_t variant);

/* The variant an E-step on (model, batch, prec) would take now, and the
 * number of variants of its route (either pointer may be NULL). */
hmm_status hmm_get_variant(const hmm_model *model, const hmm_batch *batch, hmm_precision prec,
                           int32_t *variant, int32_t *n_variants);

/* Kernel timing (tracing).  While enabled, every kernel the library enqueues
 * on this thread is bracketed by two hipEvents recorded on its stream; the
 * records accumulate until hmm_profile_reset (or re-enabling).  Record i
 * gives the kernel's name (static storage) and its elapsed milliseconds;
 * hmm_profile_get waits for that record's closing event.  Disabled by default;
 * when disabled no events are recorded. */
hmm_status hmm_profile_enable(int32_t on);
int32_t hmm_profile_count(void);
hmm_status hmm_profile_get(int32_t i, const char **name, float *ms);
hmm_status hmm_profile_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* HMM_GPU_H */
