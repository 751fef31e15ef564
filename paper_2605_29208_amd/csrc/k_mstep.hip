// k_mstep.hip -- weighted M-steps (section 4) on the device, FP64, from the
// pooled statistics of an E-step (layout of hmm_stats_len).
//
//   transitions  pi_i = sum_b gamma_1^b(i) / sum_i(.),  a_ij = Xi_ij / sum_j Xi_ij;
//                a row whose expected count is below eps keeps its old values
//   Gaussian     mu = ybar, var = N_j^-1 sum g (y - mu)^2              (4.1)
//   Poisson      lambda = ybar                                        (4.1)
//   Gamma        Newton on log a - psi(a) - c = 0 from the moment seed,
//                rate = a / ybar                                      (4.2)
//   Student-t    CM-1: mu = sum g u y / sum g u, var = sum g u (y-mu)^2 / N_j;
//                CM-2: Newton on dQ/dnu, with the expected log-mixing term
//                N_j [psi((nu+1)/2) - log((nu+1)/2)] unless the printed score
//                is requested                                         (4.3)
//   diagonal     D independent Gaussian updates                       (4.5)
//   full         mu = ybar, Sigma = weighted scatter + ridge I, L = chol(Sigma) (4.5)
// A state with N_j < eps keeps its parameters (4.4).  The statistics hold
// moments shifted by the current location, so the new location is the old
// one plus the weighted mean shift.
#include <math.h>

#include "dev_common.hpp"
#include "hmm_internal.hpp"

namespace hmmk {

// digamma and trigamma: upward recurrence to x >= 8, then the asymptotic
// series in 1/x^2 with Bernoulli-number coefficients
__device__ double dev_digamma(double x) {
    double acc = 0.0;
    while (x < 8.0) {
        acc -= 1.0 / x;
        x += 1.0;
    }
    const double r = 1.0 / x, r2 = r * r;
    const double s = r2 * (1.0 / 12 - r2 * (1.0 / 120 - r2 * (1.0 / 252 - r2 * (1.0 / 240 -
                     r2 * (1.0 / 132 - r2 * (691.0 / 32760 - r2 * (1.0 / 12)))))));
    return acc + log(x) - 0.5 * r - s;
}

__device__ double dev_trigamma(double x) {
    double acc = 0.0;
    while (x < 8.0) {
        acc += 1.0 / (x * x);
        x += 1.0;
    }
    const double r = 1.0 / x, r2 = r * r;
    const double s = r * r2 * (1.0 / 6 - r2 * (1.0 / 30 - r2 * (1.0 / 42 - r2 * (1.0 / 30 -
                     r2 * (5.0 / 66 - r2 * (691.0 / 2730 - r2 * (7.0 / 6)))))));
    return acc + r + 0.5 * r2 + s;
}

struct MLayout {
    int N, D, K;
    int64_t g1, xi, gs, fam;   // offsets into the statistics vector
};

__host__ __device__ inline MLayout mlayout(int N, int D, int K) {
    MLayout l;
    l.N = N;
    l.D = D;
    l.K = K;
    l.g1 = 1;
    l.xi = 1 + N;
    l.gs = 1 + N + (int64_t)N * N;
    l.fam = 1 + 2 * N + (int64_t)N * N;
    return l;
}

__global__ __launch_bounds__(BLOCK) void k_mstep_trans(int N, const double *__restrict__ stats,
                                                      const double *log_A_in, double eps,
                                                      double *log_pi_out, double *log_A_out) {
    const MLayout l = mlayout(N, 1, 0);
    for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < N; i += blockDim.x * gridDim.x) {
        double s = 0.0;
        for (int k = 0; k < N; ++k) s += stats[l.g1 + k];
        log_pi_out[i] = log(stats[l.g1 + i] / s);
        double r = 0.0;
        for (int j = 0; j < N; ++j) r += stats[l.xi + (int64_t)i * N + j];
        if (r < eps) {
            for (int j = 0; j < N; ++j) log_A_out[(int64_t)i * N + j] = log_A_in[(int64_t)i * N + j];
        } else {
            for (int j = 0; j < N; ++j)
                log_A_out[(int64_t)i * N + j] = log(stats[l.xi + (int64_t)i * N + j] / r);
        }
    }
}

// one thread per state for the scalar and diagonal families
__global__ __launch_bounds__(BLOCK) void k_mstep_scalar(int family, int N, int D,
                                                       const double *theta_in,
                                                       const double *__restrict__ stats,
                                                       hmm_mstep_opts o, double *theta_out,
                                                       int32_t *collapsed, int32_t *iters) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    int K = family == HMM_GAUSSIAN ? 2 : family == HMM_GAMMA ? 3 : family == HMM_STUDENT_T ? 4
          : family == HMM_POISSON ? 1 : 2 * D;
    const MLayout l = mlayout(N, D, K);
    const double Nj = stats[l.gs + j];
    const double *f = stats + l.fam + (int64_t)j * K;
    int col = 0, it = 0;
    if (!(Nj >= o.eps_collapse)) {
        col = 1;
    } else if (family == HMM_GAUSSIAN) {
        const double mu0 = theta_in[j];
        const double m1 = f[0] / Nj;
        const double var = f[1] / Nj - m1 * m1;
        theta_out[j] = mu0 + m1;
        theta_out[N + j] = var;
    } else if (family == HMM_POISSON) {
        theta_out[j] = f[0] / Nj;
    } else if (family == HMM_GAMMA) {
        const double ybar = f[0] / Nj, mlog = f[1] / Nj;
        const double c = log(ybar) - mlog;
        if (!(c > 1e-14)) {
            col = 2;
        } else {
            const double var = f[2] / Nj - ybar * ybar;
            double a = ybar * ybar / var;
            if (!(a > 0.0) || !isfinite(a))
                a = (3.0 - c + sqrt((c - 3.0) * (c - 3.0) + 24.0 * c)) / (12.0 * c);
            for (it = 0; it < o.max_iter;) {
                const double s = log(a) - dev_digamma(a) - c;
                const double ds = 1.0 / a - dev_trigamma(a);
                double step = s / ds;
                double an = a - step;
                while (!(an > 0.0)) {
                    step *= 0.5;
                    an = a - step;
                }
                const double delta = fabs(an - a);
                a = an;
                ++it;
                if (delta <= o.gamma_rtol * a) break;
            }
            theta_out[j] = a;
            theta_out[N + j] = a / ybar;
        }
    } else if (family == HMM_STUDENT_T) {
        const double mu0 = theta_in[j], nu0 = theta_in[2 * N + j];
        const double su = f[0], sud = f[1], sudd = f[2], slu = f[3];
        const double dm = sud / su;
        const double var = (sudd - sud * sud / su) / Nj;
        const double corr = o.t_nu_printed ? 0.0
                            : Nj * (dev_digamma(0.5 * (nu0 + 1.0)) - log(0.5 * (nu0 + 1.0)));
        double nu = nu0;
        for (it = 0; it < o.max_iter;) {
            const double hlf = 0.5 * nu;
            const double score = 0.5 * Nj * (log(hlf) + 1.0 - dev_digamma(hlf)) + 0.5 * (slu + corr);
            const double hess = 0.25 * Nj * (2.0 / nu - dev_trigamma(hlf));
            double step = score / hess;
            double nn = nu - step;
            while (!(nn > 0.0)) {
                step *= 0.5;
                nn = nu - step;
            }
            nn = fmin(fmax(nn, o.nu_min), o.nu_max);
            const double delta = fabs(nn - nu);
            nu = nn;
            ++it;
            if (delta < o.nu_tol) break;
        }
        theta_out[j] = mu0 + dm;
        theta_out[N + j] = sqrt(var);
        theta_out[2 * N + j] = nu;
    } else {   // diagonal Gaussian
        for (int d = 0; d < D; ++d) {
            const double m1 = f[d] / Nj;
            const double mu0 = theta_in[(int64_t)j * D + d];
            theta_out[(int64_t)j * D + d] = mu0 + m1;
            theta_out[(int64_t)N * D + (int64_t)j * D + d] = f[D + d] / Nj - m1 * m1;
        }
    }
    if (collapsed) collapsed[j] = col;
    if (iters) iters[j] = it;
}

// full covariance: one block of 64 threads per state, covariance in LDS,
// right-looking Cholesky
__global__ __launch_bounds__(64) void k_mstep_full(int N, int D, const double *theta_in,
                                                  const double *__restrict__ stats,
                                                  hmm_mstep_opts o, double *theta_out,
                                                  int32_t *collapsed, int32_t *iters) {
    __shared__ double S[64][65];
    __shared__ double m1[64];
    __shared__ int fail;
    const int j = blockIdx.x;
    const int tid = threadIdx.x;
    const int K = D + D * (D + 1) / 2;
    const MLayout l = mlayout(N, D, K);
    const double Nj = stats[l.gs + j];
    const double *f = stats + l.fam + (int64_t)j * K;
    if (!(Nj >= o.eps_collapse)) {
        if (tid == 0) {
            if (collapsed) collapsed[j] = 1;
            if (iters) iters[j] = 0;
        }
        return;
    }
    for (int d = tid; d < D; d += 64) m1[d] = f[d] / Nj;
    if (tid == 0) fail = 0;
    __syncthreads();
    for (int r = tid; r < D; r += 64) {
        int p = D + r * (r + 1) / 2;
        for (int c = 0; c <= r; ++c) {
            double v = f[p + c] / Nj - m1[r] * m1[c];
            if (r == c) v += o.ridge;
            S[r][c] = v;
        }
    }
    __syncthreads();
    for (int k = 0; k < D; ++k) {
        if (tid == 0) {
            double v = S[k][k];
            if (!(v > 0.0)) fail = 1;
            S[k][k] = sqrt(fmax(v, 0.0));
        }
        __syncthreads();
        const double lkk = S[k][k];
        for (int i = k + 1 + tid; i < D; i += 64) S[i][k] = (lkk > 0.0) ? S[i][k] / lkk : 0.0;
        __syncthreads();
        for (int i = k + 1 + tid; i < D; i += 64)
            for (int c = k + 1; c <= i; ++c) S[i][c] -= S[i][k] * S[c][k];
        __syncthreads();
    }
    if (fail) {
        if (tid == 0) {
            if (collapsed) collapsed[j] = 3;
            if (iters) iters[j] = 0;
        }
        return;
    }
    for (int d = tid; d < D; d += 64) {
        const double mu0 = theta_in[(int64_t)j * D + d];
        theta_out[(int64_t)j * D + d] = mu0 + m1[d];
    }
    double *L = theta_out + (int64_t)N * D + (int64_t)j * D * D;
    for (int k = tid; k < D * D; k += 64) {
        const int r = k / D, c = k % D;
        L[k] = (c <= r) ? S[r][c] : 0.0;
    }
    if (tid == 0) {
        if (collapsed) collapsed[j] = 0;
        if (iters) iters[j] = 0;
    }
}

void launch_mstep_trans(int N, const double *stats, const double *log_A_in, double eps,
                        double *log_pi_out, double *log_A_out, hipStream_t s) {
    ProfScope ps("mstep_transitions", s);
    hipLaunchKernelGGL(k_mstep_trans, dim3((N + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, N, stats,
                       log_A_in, eps, log_pi_out, log_A_out);
}

void launch_mstep_emission(int family, int N, int D, const double *theta_in,
                           const double *stats, const hmm_mstep_opts &o, double *theta_out,
                           int32_t *collapsed, int32_t *iters, hipStream_t s) {
    ProfScope ps("mstep_emission", s);
    if (family == HMM_FULL_GAUSSIAN)
        hipLaunchKernelGGL(k_mstep_full, dim3(N), dim3(64), 0, s, N, D, theta_in, stats, o,
                           theta_out, collapsed, iters);
    else
        hipLaunchKernelGGL(k_mstep_scalar, dim3((N + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, family,
                           N, D, theta_in, stats, o, theta_out, collapsed, iters);
}

}  // namespace hmmk
