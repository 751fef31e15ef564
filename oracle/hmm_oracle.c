/*
 * hmm_oracle.c -- plain, slow, FP64 CPU oracle for hidden-Markov-model
 * inference: emission log-densities, log-space forward-backward, posteriors,
 * pooled E-step statistics, Viterbi, posterior decoding and the weighted
 * M-steps.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is built and called by the test
 * suite, the smoke check and the benchmark's CPU-baseline leg.  The GPU
 * library never includes, links or calls it, and it shares no code, header
 * or constant table with the GPU library.
 *
 * Everything is written the direct way, following the paper's notation
 * (lambda = (pi, A, B), observations y_1..y_T; section 3.1):
 *   - log-sum-exp is the paper's definition, lse(x) = max x + log sum exp(x - max x)
 *     (section 3.2), evaluated term by term with no reformulation;
 *   - the forward recursion is eq. (loginit)/(logrec) of section 3.2;
 *   - the backward recursion, gamma and xi (section 3.2 says only that they
 *     are computed "analogously") follow the standard definitions of
 *     section 3.1: gamma_t(i) = P(q_t = i | y), xi_t(i,j) = P(q_t = i,
 *     q_{t+1} = j | y);
 *   - Viterbi is the max-plus recursion of section 3.3;
 *   - M-steps follow section 4 (closed forms 4.1, Gamma Newton 4.2,
 *     Student-t ECM 4.3, collapse guard 4.4, multivariate 4.5).
 * Sums over time steps and over sequences use Neumaier compensated
 * summation.  Nothing is fused, blocked or reordered.
 *
 * Parity status of each function is stated in the test suite; every
 * function here is pinned by at least one independent check (brute-force
 * path enumeration, scipy densities, closed forms, invariants).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* family codes (the oracle's own numbering; the Python wrapper maps names) */
enum { OF_GAUSSIAN = 0, OF_GAMMA = 1, OF_STUDENT_T = 2, OF_POISSON = 3,
       OF_DIAG = 4, OF_FULL = 5, OF_TABLE = 6 };

/* ------------------------------------------------------------------ */
/* Neumaier compensated summation                                      */
/* ------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;

static void ns_add(nsum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double ns_get(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* log-sum-exp exactly as defined in section 3.2; all -inf -> -inf       */
/* ------------------------------------------------------------------ */
double oracle_lse(const double *x, int n) {
    double m = -INFINITY;
    for (int k = 0; k < n; ++k) if (x[k] > m) m = x[k];
    if (m == -INFINITY) return -INFINITY;
    nsum s = {0, 0};
    for (int k = 0; k < n; ++k) ns_add(&s, exp(x[k] - m));
    return m + log(ns_get(&s));
}

/* ------------------------------------------------------------------ */
/* digamma and trigamma: upward recurrence to x >= shift, then the      */
/* asymptotic (Bernoulli-number) series.                                */
/*   psi(x)  = psi(x+1) - 1/x                                           */
/*   psi'(x) = psi'(x+1) + 1/x^2                                        */
/*   psi(x)  ~ ln x - 1/(2x) - sum_k B_{2k} / (2k x^{2k})                */
/*   psi'(x) ~ 1/x + 1/(2x^2) + sum_k B_{2k} / x^{2k+1}                   */
/* ------------------------------------------------------------------ */
double oracle_digamma(double x) {
    if (!(x > 0)) return NAN;
    double acc = 0.0;
    while (x < 10.0) { acc -= 1.0 / x; x += 1.0; }
    double r = 1.0 / x, r2 = r * r;
    /* B2=1/6, B4=-1/30, B6=1/42, B8=-1/30, B10=5/66, B12=-691/2730, B14=7/6 */
    double series = r2 * (1.0 / 12.0 - r2 * (1.0 / 120.0 - r2 * (1.0 / 252.0 - r2 * (1.0 / 240.0
                    - r2 * (1.0 / 132.0 - r2 * (691.0 / 32760.0 - r2 * (1.0 / 12.0)))))));
    return acc + log(x) - 0.5 * r - series;
}

double oracle_trigamma(double x) {
    if (!(x > 0)) return NAN;
    double acc = 0.0;
    while (x < 10.0) { acc += 1.0 / (x * x); x += 1.0; }
    double r = 1.0 / x, r2 = r * r;
    double series = r * r2 * (1.0 / 6.0 - r2 * (1.0 / 30.0 - r2 * (1.0 / 42.0 - r2 * (1.0 / 30.0
                    - r2 * (5.0 / 66.0 - r2 * (691.0 / 2730.0 - r2 * (7.0 / 6.0)))))));
    return acc + r + 0.5 * r2 + series;
}

/* ------------------------------------------------------------------ */
/* emission log-densities log b_j(y_t)                                  */
/* ------------------------------------------------------------------ */
static const double LOG_2PI = 1.8378770664093454835606594728112;

static double gauss_logpdf(double y, double mu, double var) {
    double d = y - mu;
    return -0.5 * log(2.0 * M_PI * var) - d * d / (2.0 * var);
}

/* log b_j(y) for one state j and one observation y (D values) */
static double emission_one(int family, int N, int D, const double *theta, int j,
                           const double *y) {
    switch (family) {
    case OF_GAUSSIAN:
        return gauss_logpdf(y[0], theta[j], theta[N + j]);
    case OF_GAMMA: {            /* shape alpha, rate beta: section 4.2 density */
        double a = theta[j], b = theta[N + j], v = y[0];
        if (!(v > 0)) return -INFINITY;
        return a * log(b) - lgamma(a) + (a - 1.0) * log(v) - b * v;
    }
    case OF_STUDENT_T: {        /* location-scale t, the scale mixture of section 4.3 */
        double mu = theta[j], s = theta[N + j], nu = theta[2 * N + j];
        double z = (y[0] - mu) / s;
        return lgamma(0.5 * (nu + 1.0)) - lgamma(0.5 * nu) - 0.5 * log(nu * M_PI * s * s)
               - 0.5 * (nu + 1.0) * log1p(z * z / nu);
    }
    case OF_POISSON: {
        double lam = theta[j], v = y[0];
        if (!(v >= 0) || floor(v) != v) return -INFINITY;
        return v * log(lam) - lam - lgamma(v + 1.0);
    }
    case OF_DIAG: {             /* product of D Gaussians, section 4.5 */
        double s = 0.0;
        for (int d = 0; d < D; ++d)
            s += gauss_logpdf(y[d], theta[j * D + d], theta[N * D + j * D + d]);
        return s;
    }
    case OF_FULL: {             /* Cholesky form, section 4.5: L z = y - mu */
        const double *mu = theta + (size_t)j * D;
        const double *L = theta + (size_t)N * D + (size_t)j * D * D;
        double z[1024];
        double quad = 0.0, logdet = 0.0;
        if (D > 1024) return NAN;
        for (int r = 0; r < D; ++r) {
            double acc = y[r] - mu[r];
            for (int c = 0; c < r; ++c) acc -= L[r * D + c] * z[c];
            z[r] = acc / L[r * D + r];
            quad += z[r] * z[r];
            logdet += log(L[r * D + r]);
        }
        return -0.5 * D * LOG_2PI - logdet - 0.5 * quad;
    }
    default:
        return NAN;
    }
}

/* out[t*N + j] = log b_j(y_t); y is [T, D] row-major */
int oracle_emission(int family, int N, int D, const double *theta, int64_t T,
                    const double *y, double *out) {
    for (int64_t t = 0; t < T; ++t)
        for (int j = 0; j < N; ++j)
            out[t * N + j] = emission_one(family, N, D, theta, j, y + t * D);
    return 0;
}

/* ------------------------------------------------------------------ */
/* forward: alpha_1(j) = log pi_j + log b_j(y_1)                         */
/*          alpha_t(j) = lse_i[alpha_{t-1}(i) + log a_ij] + log b_j(y_t)  */
/* ------------------------------------------------------------------ */
int oracle_forward(int N, const double *log_pi, const double *log_A, int64_t T,
                   const double *logB, double *alpha) {
    double *tmp = (double *)malloc(sizeof(double) * N);
    for (int j = 0; j < N; ++j) alpha[j] = log_pi[j] + logB[j];
    for (int64_t t = 1; t < T; ++t)
        for (int j = 0; j < N; ++j) {
            for (int i = 0; i < N; ++i) tmp[i] = alpha[(t - 1) * N + i] + log_A[i * N + j];
            alpha[t * N + j] = oracle_lse(tmp, N) + logB[t * N + j];
        }
    free(tmp);
    return 0;
}

/* backward: beta_T(i) = 0;
 * beta_t(i) = lse_j[log a_ij + log b_j(y_{t+1}) + beta_{t+1}(j)] */
int oracle_backward(int N, const double *log_A, int64_t T, const double *logB,
                    double *beta) {
    double *tmp = (double *)malloc(sizeof(double) * N);
    for (int i = 0; i < N; ++i) beta[(T - 1) * N + i] = 0.0;
    for (int64_t t = T - 2; t >= 0; --t)
        for (int i = 0; i < N; ++i) {
            for (int j = 0; j < N; ++j)
                tmp[j] = log_A[i * N + j] + logB[(t + 1) * N + j] + beta[(t + 1) * N + j];
            beta[t * N + i] = oracle_lse(tmp, N);
        }
    free(tmp);
    return 0;
}

/* gamma_t(i) = exp(alpha_t(i) + beta_t(i) - logL)
 * xi_t(i,j)  = exp(alpha_t(i) + log a_ij + log b_j(y_{t+1}) + beta_{t+1}(j) - logL)
 * xi (optional) is [(T-1), N, N]; xi_sum (optional) is [N, N] summed over t. */
int oracle_posteriors(int N, const double *log_A, int64_t T, const double *logB,
                      const double *alpha, const double *beta, double logL,
                      double *gamma, double *xi, double *xi_sum) {
    for (int64_t t = 0; t < T; ++t)
        for (int i = 0; i < N; ++i)
            gamma[t * N + i] = exp(alpha[t * N + i] + beta[t * N + i] - logL);
    if (!xi && !xi_sum) return 0;
    nsum *acc = (nsum *)calloc((size_t)N * N, sizeof(nsum));
    for (int64_t t = 0; t + 1 < T; ++t)
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                double v = exp(alpha[t * N + i] + log_A[i * N + j] + logB[(t + 1) * N + j]
                               + beta[(t + 1) * N + j] - logL);
                if (xi) xi[(t * N + i) * N + j] = v;
                ns_add(&acc[i * N + j], v);
            }
    if (xi_sum)
        for (int k = 0; k < N * N; ++k) xi_sum[k] = ns_get(&acc[k]);
    free(acc);
    return 0;
}

/* ------------------------------------------------------------------ */
/* pooled E-step statistics                                             */
/*   [ sum_b logL_b | sum_b gamma_1 (N) | sum_b sum_t xi_t (N*N) |        */
/*     sum gamma (N) | family block (N x K) ]                            */
/* family block, per state j, with d = y - (current location):          */
/*   gaussian  K=2   sum g d, sum g d^2                        (d = y - mu_j)  */
/*   gamma     K=3   sum g y, sum g log y, sum g y^2                       */
/*   student-t K=4   sum g u, sum g u d, sum g u d^2, sum g (log u - u)     */
/*                   with u = (nu+1)/(nu + d^2/sigma^2), eq. (utilde)       */
/*   poisson   K=1   sum g y                                             */
/*   diag      K=2D  [sum g d_k]_k, [sum g d_k^2]_k            (d = y - mu_j)  */
/*   full      K=D+D(D+1)/2  [sum g d_k]_k, packed lower [sum g d_r d_c]_{r>=c} */
/*   table     K=0   (emission given as a table; no family statistics)   */
/* ------------------------------------------------------------------ */
static int family_k(int family, int D) {
    switch (family) {
    case OF_GAUSSIAN: return 2;
    case OF_GAMMA: return 3;
    case OF_STUDENT_T: return 4;
    case OF_POISSON: return 1;
    case OF_DIAG: return 2 * D;
    case OF_FULL: return D + D * (D + 1) / 2;
    case OF_TABLE: return 0;
    default: return -1;
    }
}

int64_t oracle_stats_len(int family, int N, int D) {
    int k = family_k(family, D);
    if (k < 0) return -1;
    return 1 + (int64_t)N + (int64_t)N * N + N + (int64_t)N * k;
}

static void family_terms(int family, int N, int D, const double *theta, int j,
                         const double *y, double *out /* K values */) {
    switch (family) {
    case OF_GAUSSIAN: {
        double d = y[0] - theta[j];
        out[0] = d; out[1] = d * d; break;
    }
    case OF_GAMMA:
        out[0] = y[0]; out[1] = log(y[0]); out[2] = y[0] * y[0]; break;
    case OF_STUDENT_T: {
        double mu = theta[j], s = theta[N + j], nu = theta[2 * N + j];
        double d = y[0] - mu;
        double u = (nu + 1.0) / (nu + d * d / (s * s));
        out[0] = u; out[1] = u * d; out[2] = u * d * d; out[3] = log(u) - u; break;
    }
    case OF_POISSON:
        out[0] = y[0]; break;
    case OF_DIAG:
        for (int k = 0; k < D; ++k) {
            double d = y[k] - theta[j * D + k];
            out[k] = d; out[D + k] = d * d;
        }
        break;
    case OF_FULL: {
        const double *mu = theta + (size_t)j * D;
        for (int k = 0; k < D; ++k) out[k] = y[k] - mu[k];
        int p = D;
        for (int r = 0; r < D; ++r)
            for (int c = 0; c <= r; ++c) out[p++] = out[r] * out[c];
        break;
    }
    default: break;
    }
}

/*
 * One E-step over B sequences.  obs is [sum T, D]; offsets [B+1].
 * If logB_in is non-NULL it supplies log b_j(y_t) as a [sum T, N] table and
 * obs is only used for the family statistics (may be NULL for OF_TABLE).
 * Outputs: stats [oracle_stats_len], loglik[B], loglik_bwd[B] (optional),
 * status[B]: 0 ok, 1 logL = -inf, 2 non-finite observation (sequence skipped),
 * 3 empty sequence.  gamma_out (optional) is [sum T, N].
 * Returns 0, or -1 for bad arguments.
 */
int oracle_estep(int family, int N, int D, const double *log_pi, const double *log_A,
                 const double *theta, int64_t B, const int64_t *offsets, const double *obs,
                 const double *logB_in, double *stats, double *loglik, double *loglik_bwd,
                 int32_t *status, double *gamma_out) {
    int K = family_k(family, D);
    if (K < 0 || N <= 0) return -1;
    int64_t len = oracle_stats_len(family, N, D);
    nsum *acc = (nsum *)calloc((size_t)len, sizeof(nsum));
    double *fam = (double *)malloc(sizeof(double) * (K > 0 ? K : 1));
    for (int64_t b = 0; b < B; ++b) {
        int64_t o = offsets[b], T = offsets[b + 1] - offsets[b];
        status[b] = 0;
        loglik[b] = NAN;
        if (loglik_bwd) loglik_bwd[b] = NAN;
        if (T <= 0) { status[b] = 3; continue; }
        int bad = 0;
        if (obs)
            for (int64_t k = 0; k < T * D; ++k) if (!isfinite(obs[o * D + k])) bad = 1;
        if (logB_in)
            for (int64_t k = 0; k < T * N; ++k) if (isnan(logB_in[o * N + k])) bad = 1;
        if (bad) { status[b] = 2; continue; }
        double *logB = (double *)malloc(sizeof(double) * T * N);
        double *alpha = (double *)malloc(sizeof(double) * T * N);
        double *beta = (double *)malloc(sizeof(double) * T * N);
        double *gamma = (double *)malloc(sizeof(double) * T * N);
        double *xis = (double *)malloc(sizeof(double) * N * N);
        if (logB_in) memcpy(logB, logB_in + o * N, sizeof(double) * T * N);
        else oracle_emission(family, N, D, theta, T, obs + o * D, logB);
        oracle_forward(N, log_pi, log_A, T, logB, alpha);
        oracle_backward(N, log_A, T, logB, beta);
        double ll = oracle_lse(alpha + (T - 1) * N, N);
        double *tmp = (double *)malloc(sizeof(double) * N);
        for (int j = 0; j < N; ++j) tmp[j] = log_pi[j] + logB[j] + beta[j];
        double ll2 = oracle_lse(tmp, N);
        free(tmp);
        loglik[b] = ll;
        if (loglik_bwd) loglik_bwd[b] = ll2;
        if (ll == -INFINITY) {
            status[b] = 1;
        } else {
            oracle_posteriors(N, log_A, T, logB, alpha, beta, ll, gamma, NULL, xis);
            ns_add(&acc[0], ll);
            for (int i = 0; i < N; ++i) ns_add(&acc[1 + i], gamma[i]);
            for (int k = 0; k < N * N; ++k) ns_add(&acc[1 + N + k], xis[k]);
            for (int64_t t = 0; t < T; ++t)
                for (int j = 0; j < N; ++j) {
                    double g = gamma[t * N + j];
                    ns_add(&acc[1 + N + N * N + j], g);
                    if (K > 0) {
                        family_terms(family, N, D, theta, j, obs + (o + t) * D, fam);
                        for (int k = 0; k < K; ++k)
                            ns_add(&acc[1 + 2 * N + N * N + (int64_t)j * K + k], g * fam[k]);
                    }
                }
            if (gamma_out) memcpy(gamma_out + o * N, gamma, sizeof(double) * T * N);
        }
        free(logB); free(alpha); free(beta); free(gamma); free(xis);
    }
    for (int64_t k = 0; k < len; ++k) stats[k] = ns_get(&acc[k]);
    free(acc);
    free(fam);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Viterbi (section 3.3): delta_1 = log pi + log b(y_1);                  */
/* delta_t(j) = max_i[delta_{t-1}(i) + log a_ij] + log b_j(y_t);          */
/* psi_t(j) = the lowest i attaining the max.  Each step is shifted by    */
/* max_j delta_t(j) (an exact shift for the argmax), with the shift       */
/* summed into the path score.  A decision is a tie when the best and     */
/* second-best candidates differ by less than tie_eps.                   */
/* path [T], returns the path log-probability in *logp and the number of   */
/* near-ties met along the returned path in *n_ties.                      */
/* ------------------------------------------------------------------ */
int oracle_viterbi(int N, const double *log_pi, const double *log_A, int64_t T,
                   const double *logB, double tie_eps, int32_t *path, double *logp,
                   int32_t *n_ties) {
    double *delta = (double *)malloc(sizeof(double) * N);
    double *nd = (double *)malloc(sizeof(double) * N);
    int32_t *psi = (int32_t *)malloc(sizeof(int32_t) * T * N);
    double *gap = (double *)malloc(sizeof(double) * T * N);
    double offset = 0.0;
    for (int j = 0; j < N; ++j) delta[j] = log_pi[j] + logB[j];
    double m = -INFINITY;
    for (int j = 0; j < N; ++j) if (delta[j] > m) m = delta[j];
    if (m == -INFINITY) {
        for (int64_t t = 0; t < T; ++t) path[t] = -1;
        *logp = -INFINITY; *n_ties = 0;
        free(delta); free(nd); free(psi); free(gap);
        return 1;
    }
    for (int j = 0; j < N; ++j) delta[j] -= m;
    offset += m;
    for (int64_t t = 1; t < T; ++t) {
        for (int j = 0; j < N; ++j) {
            double best = -INFINITY, second = -INFINITY;
            int arg = 0;
            for (int i = 0; i < N; ++i) {
                double v = delta[i] + log_A[i * N + j];
                if (v > best) { second = best; best = v; arg = i; }
                else if (v > second) second = v;
            }
            psi[t * N + j] = arg;
            gap[t * N + j] = best - second;
            nd[j] = best + logB[t * N + j];
        }
        m = -INFINITY;
        for (int j = 0; j < N; ++j) if (nd[j] > m) m = nd[j];
        if (m == -INFINITY) {
            for (int64_t k = 0; k < T; ++k) path[k] = -1;
            *logp = -INFINITY; *n_ties = 0;
            free(delta); free(nd); free(psi); free(gap);
            return 1;
        }
        for (int j = 0; j < N; ++j) delta[j] = nd[j] - m;
        offset += m;
    }
    int q = 0;
    double best = -INFINITY, second = -INFINITY;
    for (int j = 0; j < N; ++j) {
        if (delta[j] > best) { second = best; best = delta[j]; q = j; }
        else if (delta[j] > second) second = delta[j];
    }
    int ties = (best - second < tie_eps) ? 1 : 0;
    *logp = offset + best;
    path[T - 1] = q;
    for (int64_t t = T - 1; t >= 1; --t) {
        if (gap[t * N + q] < tie_eps) ++ties;
        q = psi[t * N + q];
        path[t - 1] = q;
    }
    *n_ties = ties;
    free(delta); free(nd); free(psi); free(gap);
    return 0;
}

/* posterior decoding (section 3.4): q_t = lowest argmax_j gamma_t(j) */
int oracle_posterior_decode(int N, int64_t T, const double *gamma, int32_t *path) {
    for (int64_t t = 0; t < T; ++t) {
        int q = 0;
        for (int j = 1; j < N; ++j) if (gamma[t * N + j] > gamma[t * N + q]) q = j;
        path[t] = q;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* M-steps (section 4).  All read the pooled statistics of oracle_estep. */
/* ------------------------------------------------------------------ */

/* pi_i = sum_b gamma_1^b(i) / sum_i(.);  a_ij = Xi_ij / sum_j Xi_ij.
 * A row whose expected transition count is below eps keeps its old values. */
int oracle_mstep_transitions(int N, const double *stats, const double *log_A_old,
                             double eps, double *log_pi_out, double *log_A_out,
                             int32_t *row_kept) {
    const double *g1 = stats + 1, *xi = stats + 1 + N;
    double s = 0;
    for (int i = 0; i < N; ++i) s += g1[i];
    for (int i = 0; i < N; ++i) log_pi_out[i] = log(g1[i] / s);
    for (int i = 0; i < N; ++i) {
        double r = 0;
        for (int j = 0; j < N; ++j) r += xi[i * N + j];
        row_kept[i] = r < eps;
        for (int j = 0; j < N; ++j)
            log_A_out[i * N + j] = (r < eps) ? log_A_old[i * N + j] : log(xi[i * N + j] / r);
    }
    return 0;
}

/* options of the emission M-steps */
typedef struct {
    double eps_collapse;   /* N_j below this keeps theta_j (section 4.4): 1e-8 */
    double ridge;          /* full covariance + ridge * I (section 4.5): 1e-6 */
    double gamma_rtol;     /* Gamma Newton stop |d alpha| <= rtol * alpha: 1e-12 */
    double nu_tol;         /* Student-t Newton stop |d nu| < tol (section 4.3): 1e-6 */
    double nu_min, nu_max; /* clamp of nu: 0.5, 1e4 */
    int32_t max_iter;      /* 100 */
    int32_t t_nu_printed;  /* 1: use the score exactly as printed (no E[log U] term) */
} oracle_mopts;

/* Gamma shape: Newton on s(a) = log a - psi(a) - c (section 4.2) from the
 * moment seed a0 = ybar^2 / var.  Returns the number of iterations. */
static int gamma_newton(double c, double a0, double rtol, int max_iter, double *a_out) {
    double a = a0;
    int it = 0;
    for (; it < max_iter; ++it) {
        double s = log(a) - oracle_digamma(a) - c;
        double ds = 1.0 / a - oracle_trigamma(a);
        double step = s / ds;
        double an = a - step;
        while (!(an > 0)) { step *= 0.5; an = a - step; }
        double delta = fabs(an - a);
        a = an;
        if (delta <= rtol * a) { ++it; break; }
    }
    *a_out = a;
    return it;
}

/* Student-t degrees of freedom, Newton on dQ/dnu (section 4.3).
 * sum_lu = sum_t gamma (log u - u); with the correction (default) the
 * expected log-mixing term N [psi((nu_old+1)/2) - log((nu_old+1)/2)] is added. */
static int t_nu_newton(double Nj, double sum_lu, double nu_old, const oracle_mopts *o,
                       double *nu_out) {
    double corr = o->t_nu_printed ? 0.0
                  : Nj * (oracle_digamma(0.5 * (nu_old + 1.0)) - log(0.5 * (nu_old + 1.0)));
    double nu = nu_old;
    int it = 0;
    for (; it < o->max_iter; ++it) {
        double h = 0.5 * nu;
        double score = 0.5 * Nj * (log(h) + 1.0 - oracle_digamma(h)) + 0.5 * (sum_lu + corr);
        double hess = 0.25 * Nj * (2.0 / nu - oracle_trigamma(h));
        double step = score / hess;
        double nn = nu - step;
        while (!(nn > 0)) { step *= 0.5; nn = nu - step; }
        if (nn < o->nu_min) nn = o->nu_min;
        if (nn > o->nu_max) nn = o->nu_max;
        double delta = fabs(nn - nu);
        nu = nn;
        if (delta < o->nu_tol) { ++it; break; }
    }
    *nu_out = nu;
    return it;
}

/* in-place Cholesky of a [D, D] SPD matrix (lower, row-major); returns 0 or -1 */
static int cholesky(int D, double *a) {
    for (int j = 0; j < D; ++j) {
        double s = a[j * D + j];
        for (int k = 0; k < j; ++k) s -= a[j * D + k] * a[j * D + k];
        if (!(s > 0)) return -1;
        double l = sqrt(s);
        a[j * D + j] = l;
        for (int i = j + 1; i < D; ++i) {
            double v = a[i * D + j];
            for (int k = 0; k < j; ++k) v -= a[i * D + k] * a[j * D + k];
            a[i * D + j] = v / l;
        }
        for (int k = j + 1; k < D; ++k) a[j * D + k] = 0.0;
    }
    return 0;
}

/*
 * Emission M-step for every state, from pooled statistics and the current
 * parameters theta_old (the location shift of the statistics).
 * collapsed[j] = 1 when N_j < eps (parameters kept); 2 when the Gamma
 * statistic c_j <= 1e-14 (all observations equal; parameters kept);
 * 3 when a covariance was not positive definite (kept).
 * iters[j] = Newton iterations used (Gamma shape or t degrees of freedom).
 * Returns 0, or -1 for an unsupported family.
 */
int oracle_mstep_emission(int family, int N, int D, const double *theta_old,
                          const double *stats, const oracle_mopts *o, double *theta,
                          int32_t *collapsed, int32_t *iters) {
    int K = family_k(family, D);
    if (K <= 0) return -1;
    const double *Ng = stats + 1 + N + N * N;
    const double *F = stats + 1 + 2 * N + N * N;
    int64_t plen;
    switch (family) {
    case OF_GAUSSIAN: case OF_GAMMA: plen = 2 * N; break;
    case OF_STUDENT_T: plen = 3 * N; break;
    case OF_POISSON: plen = N; break;
    case OF_DIAG: plen = 2 * (int64_t)N * D; break;
    case OF_FULL: plen = (int64_t)N * D + (int64_t)N * D * D; break;
    default: return -1;
    }
    memcpy(theta, theta_old, sizeof(double) * plen);
    for (int j = 0; j < N; ++j) {
        double Nj = Ng[j];
        const double *f = F + (int64_t)j * K;
        collapsed[j] = 0;
        iters[j] = 0;
        if (!(Nj >= o->eps_collapse)) { collapsed[j] = 1; continue; }
        switch (family) {
        case OF_GAUSSIAN: {     /* mu = ybar; var = N^-1 sum g (y - mu)^2  (section 4.1) */
            double m1 = f[0] / Nj;
            theta[j] = theta_old[j] + m1;
            theta[N + j] = f[1] / Nj - m1 * m1;
            break;
        }
        case OF_GAMMA: {        /* section 4.2 */
            double ybar = f[0] / Nj, mlog = f[1] / Nj;
            double c = log(ybar) - mlog;
            if (!(c > 1e-14)) { collapsed[j] = 2; break; }
            double var = f[2] / Nj - ybar * ybar;
            double a0 = ybar * ybar / var;
            if (!(a0 > 0) || !isfinite(a0))
                a0 = (3.0 - c + sqrt((c - 3.0) * (c - 3.0) + 24.0 * c)) / (12.0 * c);
            double a;
            iters[j] = gamma_newton(c, a0, o->gamma_rtol, o->max_iter, &a);
            theta[j] = a;
            theta[N + j] = a / ybar;
            break;
        }
        case OF_STUDENT_T: {    /* ECM: CM-1 eq. (mu), (sigma); CM-2 nu Newton (section 4.3) */
            double su = f[0], sud = f[1], sudd = f[2], slu = f[3];
            double dm = sud / su;
            double mu = theta_old[j] + dm;
            double var = (sudd - sud * sud / su) / Nj;
            theta[j] = mu;
            theta[N + j] = sqrt(var);
            double nu;
            iters[j] = t_nu_newton(Nj, slu, theta_old[2 * N + j], o, &nu);
            theta[2 * N + j] = nu;
            break;
        }
        case OF_POISSON:        /* lambda = ybar (section 4.1) */
            theta[j] = f[0] / Nj;
            break;
        case OF_DIAG:           /* D independent Gaussian updates (section 4.5) */
            for (int k = 0; k < D; ++k) {
                double m1 = f[k] / Nj;
                theta[j * D + k] = theta_old[j * D + k] + m1;
                theta[N * D + j * D + k] = f[D + k] / Nj - m1 * m1;
            }
            break;
        case OF_FULL: {         /* mu = ybar; Sigma = weighted scatter + ridge I; L = chol */
            double *S = (double *)malloc(sizeof(double) * D * D);
            double *m1 = (double *)malloc(sizeof(double) * D);
            for (int k = 0; k < D; ++k) m1[k] = f[k] / Nj;
            int p = D;
            for (int r = 0; r < D; ++r)
                for (int c = 0; c <= r; ++c) {
                    double v = f[p++] / Nj - m1[r] * m1[c];
                    S[r * D + c] = v;
                    S[c * D + r] = v;
                }
            for (int k = 0; k < D; ++k) S[k * D + k] += o->ridge;
            if (cholesky(D, S) != 0) {
                collapsed[j] = 3;
            } else {
                for (int k = 0; k < D; ++k) theta[j * D + k] = theta_old[j * D + k] + m1[k];
                memcpy(theta + (int64_t)N * D + (int64_t)j * D * D, S, sizeof(double) * D * D);
            }
            free(S); free(m1);
            break;
        }
        }
    }
    return 0;
}
