// k_plain.hip -- the paper's recursion taken literally on the GPU, and the
// emission-table kernel.
//
// Plain path: one thread per sequence; the log-space forward recursion of
// section 3.2 (eq. loginit / logrec) with lse(x) = max x + log sum exp(x -
// max x) evaluated term by term (N exponentials per state per step, as the
// paper notes), the backward recursion, and gamma/xi from the definitions of
// section 3.1, each in its own kernel with alpha, beta and log b stored in
// device memory.  To keep single precision usable over long sequences every
// step is shifted by its maximum with the shifts summed in FP64.
#include "dev_common.hpp"
#include "hmm_internal.hpp"

namespace hmmk {

// emission table: one thread per (step, state)
template <typename R>
__global__ __launch_bounds__(BLOCK) void k_emission_table(StagedModel<R> m, ObsRef o,
                                                          int64_t total, R *out) {
    const int64_t idx = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= total * m.N) return;
    const int64_t row = idx / m.N;
    const int j = (int)(idx % m.N);
    double common;
    bool bad;
    double v = emission_any<R>(m, o, row, j, &common, &bad);
    out[idx] = bad ? (R)__builtin_nan("") : (R)(v + common);
}

template <typename R>
hmm_status run_emission(const StagedModel<R> &m, const ObsDesc &o, int64_t total, R *out,
                        hipStream_t s) {
    int64_t n = total * m.N;
    if (n == 0) return HMM_OK;
    ProfScope ps("emission_table", s);
    hipLaunchKernelGGL(k_emission_table<R>, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK),
                       0, s, m, ObsRef{o.obs, o.obs_f64}, total, out);
    return HMM_OK;
}
template hmm_status run_emission<float>(const StagedModel<float> &, const ObsDesc &, int64_t,
                                        float *, hipStream_t);
template hmm_status run_emission<double>(const StagedModel<double> &, const ObsDesc &, int64_t,
                                         double *, hipStream_t);

// ---- plain path kernels (thread = sequence) ----

template <typename R>
__global__ __launch_bounds__(64) void k_plain_emission(StagedModel<R> m, ObsRef o, int64_t nseq,
                                                       const int64_t *offsets, R *logB,
                                                       double *comsum, int32_t *status) {
    const int64_t b = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (b >= nseq) return;
    const int N = m.N;
    const int64_t off = offsets[b], T = offsets[b + 1] - off;
    double cs = 0.0;
    bool badany = false;
    for (int64_t t = 0; t < T; ++t) {
        // store log b shifted by its per-step maximum; the shift joins the FP64 offset
        double common = 0.0, mx = -__builtin_inf();
        for (int j = 0; j < N; ++j) {
            bool bad;
            mx = fmax(mx, emission_any<R>(m, o, off + t, j, &common, &bad));
            badany |= bad;
        }
        for (int j = 0; j < N; ++j) {
            bool bad;
            double v = emission_any<R>(m, o, off + t, j, &common, &bad);
            logB[(off + t) * N + j] = (mx == -__builtin_inf()) ? (R)v : (R)(v - mx);
        }
        cs += common + ((mx == -__builtin_inf()) ? 0.0 : mx);
    }
    comsum[b] = cs;
    status[b] = *m.perr ? 4 : (badany ? 2 : 0);
}

template <typename R>
__global__ __launch_bounds__(64) void k_plain_forward(StagedModel<R> m, int64_t nseq,
                                                      const int64_t *offsets, const R *logB,
                                                      R *alpha, const double *comsum,
                                                      double *loglik, int32_t *status) {
    const int64_t b = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (b >= nseq) return;
    const int N = m.N;
    const int64_t off = offsets[b], T = offsets[b + 1] - off;
    if (status[b] != 0) {
        loglik[b] = __builtin_nan("");
        return;
    }
    R *a = alpha + off * N;
    const R *lb = logB + off * N;
    const R ninf = neg_inf<R>();
    double C = 0.0;
    bool dead = false;
    // alpha_1(j) = log pi_j + log b_j(y_1)
    R c = ninf;
    for (int j = 0; j < N; ++j) {
        a[j] = m.lpi[j] + lb[j];
        c = fmax(c, a[j]);
    }
    if (c == ninf) dead = true;
    else {
        for (int j = 0; j < N; ++j) a[j] -= c;
        C += (double)c;
    }
    for (int64_t t = 1; t < T && !dead; ++t) {
        R cm = ninf;
        for (int j = 0; j < N; ++j) {
            // lse_i[alpha_{t-1}(i) + log a_ij]
            R mx = ninf;
            for (int i = 0; i < N; ++i) mx = fmax(mx, a[(t - 1) * N + i] + m.lA[i * N + j]);
            R v = ninf;
            if (mx != ninf) {
                R s = (R)0;
                for (int i = 0; i < N; ++i) s += fexp_e(a[(t - 1) * N + i] + m.lA[i * N + j] - mx);
                v = mx + flog(s) + lb[t * N + j];
            }
            a[t * N + j] = v;
            cm = fmax(cm, v);
        }
        if (cm == ninf) { dead = true; break; }
        for (int j = 0; j < N; ++j) a[t * N + j] -= cm;
        C += (double)cm;
    }
    if (dead) {
        loglik[b] = -__builtin_inf();
        status[b] = 1;
        return;
    }
    R mx = ninf;
    for (int j = 0; j < N; ++j) mx = fmax(mx, a[(T - 1) * N + j]);
    R s = (R)0;
    for (int j = 0; j < N; ++j) s += fexp_e(a[(T - 1) * N + j] - mx);
    loglik[b] = C + (double)mx + log((double)s) + comsum[b];
}

template <typename R>
__global__ __launch_bounds__(64) void k_plain_backward(StagedModel<R> m, int64_t nseq,
                                                       const int64_t *offsets, const R *logB,
                                                       R *beta, const int32_t *status) {
    const int64_t b = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (b >= nseq || status[b] != 0) return;
    const int N = m.N;
    const int64_t off = offsets[b], T = offsets[b + 1] - off;
    R *be = beta + off * N;
    const R *lb = logB + off * N;
    const R ninf = neg_inf<R>();
    for (int i = 0; i < N; ++i) be[(T - 1) * N + i] = (R)0;
    for (int64_t t = T - 2; t >= 0; --t) {
        R cm = ninf;
        for (int i = 0; i < N; ++i) {
            // lse_j[log a_ij + log b_j(y_{t+1}) + beta_{t+1}(j)]
            R mx = ninf;
            for (int j = 0; j < N; ++j)
                mx = fmax(mx, m.lA[i * N + j] + lb[(t + 1) * N + j] + be[(t + 1) * N + j]);
            R v = ninf;
            if (mx != ninf) {
                R s = (R)0;
                for (int j = 0; j < N; ++j)
                    s += fexp_e(m.lA[i * N + j] + lb[(t + 1) * N + j] + be[(t + 1) * N + j] - mx);
                v = mx + flog(s);
            }
            be[t * N + i] = v;
            cm = fmax(cm, v);
        }
        for (int i = 0; i < N; ++i) be[t * N + i] -= cm;
    }
}

// per-sequence statistics row ps[b*S ..], layout of hmm_stats_len
template <typename R>
__global__ __launch_bounds__(64) void k_plain_stats(StagedModel<R> m, ObsRef o, int64_t nseq,
                                                    const int64_t *offsets, const R *logB,
                                                    const R *alpha, const R *beta,
                                                    const int32_t *status, double *ps, int64_t S,
                                                    int K, R *gamma_out) {
    const int64_t b = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (b >= nseq) return;
    double *row = ps + b * S;
    for (int64_t s = 0; s < S; ++s) row[s] = 0.0;
    const int N = m.N, D = m.D;
    const int64_t off = offsets[b], T = offsets[b + 1] - off;
    if (status[b] != 0) {
        if (gamma_out)
            for (int64_t k = 0; k < T * N; ++k) gamma_out[off * N + k] = (R)0;
        return;
    }
    const R *a = alpha + off * N, *be = beta + off * N, *lb = logB + off * N;
    const R ninf = neg_inf<R>();
    // gamma_t(i) = exp(alpha + beta - lse_i(alpha + beta))
    for (int64_t t = 0; t < T; ++t) {
        R mx = ninf;
        for (int i = 0; i < N; ++i) mx = fmax(mx, a[t * N + i] + be[t * N + i]);
        R s = (R)0;
        for (int i = 0; i < N; ++i) s += fexp_e(a[t * N + i] + be[t * N + i] - mx);
        R lz = mx + flog(s);
        for (int i = 0; i < N; ++i) {
            R g = fexp_e(a[t * N + i] + be[t * N + i] - lz);
            if (gamma_out) gamma_out[(off + t) * N + i] = g;
            if (t == 0) row[1 + i] = (double)g;
            row[1 + N + (int64_t)N * N + i] += (double)g;
            // family terms
            double *f = row + 1 + 2 * N + (int64_t)N * N + (int64_t)i * K;
            switch (m.family) {
            case HMM_GAUSSIAN: {
                R d = load_obs<R>(o, off + t) - m.ep[i * EP_STRIDE];
                f[0] += (double)(g * d);
                f[1] += (double)(g * d * d);
                break;
            }
            case HMM_GAMMA: {
                R y = load_obs<R>(o, off + t);
                f[0] += (double)(g * y);
                f[1] += (double)(g * flog(y));
                f[2] += (double)(g * y * y);
                break;
            }
            case HMM_STUDENT_T: {
                const R *k = m.ep + i * EP_STRIDE;
                R d = load_obs<R>(o, off + t) - k[0];
                R u = k[4] / ((R)1 + k[1] * d * d);
                f[0] += (double)(g * u);
                f[1] += (double)(g * u * d);
                f[2] += (double)(g * u * d * d);
                f[3] += (double)(g * (flog(u) - u));
                break;
            }
            case HMM_POISSON:
                f[0] += (double)(g * load_obs<R>(o, off + t));
                break;
            case HMM_DIAG_GAUSSIAN:
                for (int d = 0; d < D; ++d) {
                    R dv = load_obs<R>(o, (off + t) * D + d) - m.mv[(size_t)i * D + d];
                    f[d] += (double)(g * dv);
                    f[D + d] += (double)(g * dv * dv);
                }
                break;
            case HMM_FULL_GAUSSIAN: {
                int pk = D;
                for (int r = 0; r < D; ++r) {
                    R dr = load_obs<R>(o, (off + t) * D + r) - m.mv[(size_t)i * D + r];
                    f[r] += (double)(g * dr);
                    for (int c = 0; c <= r; ++c) {
                        R dc = load_obs<R>(o, (off + t) * D + c) - m.mv[(size_t)i * D + c];
                        f[pk++] += (double)(g * dr * dc);
                    }
                }
                break;
            }
            default:
                break;
            }
        }
    }
    // xi_t(i,j) = exp(alpha_t(i) + log a_ij + log b_j(y_{t+1}) + beta_{t+1}(j) - lse_ij(...))
    for (int64_t t = 0; t + 1 < T; ++t) {
        R mx = ninf;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j)
                mx = fmax(mx, a[t * N + i] + m.lA[i * N + j] + lb[(t + 1) * N + j] +
                                  be[(t + 1) * N + j]);
        R s = (R)0;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j)
                s += fexp_e(a[t * N + i] + m.lA[i * N + j] + lb[(t + 1) * N + j] +
                            be[(t + 1) * N + j] - mx);
        R lz = mx + flog(s);
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j)
                row[1 + N + (int64_t)i * N + j] += (double)fexp_e(
                    a[t * N + i] + m.lA[i * N + j] + lb[(t + 1) * N + j] + be[(t + 1) * N + j] - lz);
    }
}

template <typename R>
hmm_status run_plain(const StagedModel<R> &m, const ObsDesc &o, const PlainBuffers &pb,
                     double *loglik, int32_t *status, void *gamma_out, double *stats, int64_t S,
                     hipStream_t s) {
    const unsigned nb = (unsigned)((o.nseq + 63) / 64);
    if (nb == 0) {
        if (stats) launch_reduce_stats(pb.ps, 0, S, loglik, status, 0, stats, pb.red, s);
        return HMM_OK;
    }
    ObsRef obs{o.obs, o.obs_f64};
    R *logB = (R *)pb.logB, *alpha = (R *)pb.alpha, *beta = (R *)pb.beta;
    double *csum = pb.ps + o.nseq * S;   // per-sequence sum of state-independent terms
    const int K = (int)((S - 1 - 2 * (int64_t)m.N - (int64_t)m.N * m.N) / m.N);
    {
        ProfScope ps("plain_emission", s);
        hipLaunchKernelGGL(k_plain_emission<R>, dim3(nb), dim3(64), 0, s, m, obs, o.nseq,
                           o.offsets, logB, csum, status);
    }
    {
        ProfScope ps("plain_forward", s);
        hipLaunchKernelGGL(k_plain_forward<R>, dim3(nb), dim3(64), 0, s, m, o.nseq, o.offsets,
                           (const R *)logB, alpha, (const double *)csum, loglik, status);
    }
    {
        ProfScope ps("plain_backward", s);
        hipLaunchKernelGGL(k_plain_backward<R>, dim3(nb), dim3(64), 0, s, m, o.nseq, o.offsets,
                           (const R *)logB, beta, (const int32_t *)status);
    }
    {
        ProfScope ps("plain_stats", s);
        hipLaunchKernelGGL(k_plain_stats<R>, dim3(nb), dim3(64), 0, s, m, obs, o.nseq, o.offsets,
                           (const R *)logB, (const R *)alpha, (const R *)beta,
                           (const int32_t *)status, pb.ps, S, K, (R *)gamma_out);
    }
    if (stats) launch_reduce_stats(pb.ps, (int)o.nseq, S, loglik, status, o.nseq, stats, pb.red, s);
    return HMM_OK;
}

template hmm_status run_plain<float>(const StagedModel<float> &, const ObsDesc &,
                                     const PlainBuffers &, double *, int32_t *, void *, double *,
                                     int64_t, hipStream_t);
template hmm_status run_plain<double>(const StagedModel<double> &, const ObsDesc &,
                                      const PlainBuffers &, double *, int32_t *, void *, double *,
                                      int64_t, hipStream_t);

}  // namespace hmmk
