// k_block.hip -- batched forward-backward E-step for large state counts
// (N <= 256) and for the multivariate families, one workgroup per sequence.
//
//   1. emission pass (all steps in parallel): e_t(j) = exp(log b_j(y_t) - m_t)
//      with m_t = max_j log b_j(y_t), and m_t plus the state-independent part
//      in FP64;
//   2. forward sweep (section 3.1 recursion, normalised): alpha^_t = (alpha^_{t-1} A) o e_t
//      scaled by 2^-x_t (x_t = binary exponent of its largest entry); every
//      alpha^_t row and x_t are kept, with log P(y) = sum_t m_t + ln2 sum_t x_t
//      + log sum_j alpha^_{T-1}(j);
//   3. backward sweep: beta^_{t-1} = A (e_t o beta^_t) rescaled the same way,
//      and at each step the posterior gamma_t = alpha^_t o beta^_t / Z_t
//      (Z_t = sum_j alpha^_t(j) beta^_t(j)) and
//        w'_t = e_t o beta^_t * 2^-x_t / Z_t,
//      which makes xi_t(i,j) = alpha^_{t-1}(i) a_ij w'_t(j) (the normaliser of
//      xi_t, sum_ij alpha^_{t-1}(i) a_ij e_t(j) beta^_t(j), equals 2^x_t Z_t);
//      w'_t overwrites e_t in place;
//   4. sum_t xi_t = (sum_t alpha^_{t-1}^T w'_t) o A: a dense contraction over
//      all steps of all sequences, done as one library GEMM (rows of the first
//      step of a sequence have w' = 0, so pairing row r of alpha^ with row
//      r + 1 of w' across the whole batch is exact);
//   5. gamma-weighted family sums (all steps in parallel, one thread per
//      (state, dimension)), gamma_1, and the assembly of the statistics.
//
// Sweeps: 256 threads, thread (c, p) owns column c (state) and the p-th of
// 256 / NC row blocks (NC = N rounded up to 64); partial products meet in LDS.
#include <rocblas/rocblas.h>

#include "dev_common.hpp"
#include "hmm_internal.hpp"

namespace hmmk {

constexpr int BT = 256;   // threads of the sweep and emission blocks

__device__ __forceinline__ double wave_max_dbl(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
template <typename R>
__device__ __forceinline__ R wave_sum_r(R v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename R>
__device__ __forceinline__ R wave_max_r(R v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__host__ __device__ inline int blk_nc(int N) { return ((N + 63) / 64) * 64; }

// ---------------------------------------------------------------- 1. emissions
template <typename R>
__global__ __launch_bounds__(BT) void k_blk_emit(StagedModel<R> m, ObsRef o, int64_t total,
                                                 R *__restrict__ etab, double *__restrict__ mt) {
    __shared__ double wm[BT / 64];
    __shared__ int wb[BT / 64];
    const int N = m.N, NC = blk_nc(N), SPB = BT / NC, WPS = NC / 64;
    const int c = threadIdx.x % NC, q = threadIdx.x / NC, wv = threadIdx.x / 64;
    const bool inq = q < SPB;   // threads beyond SPB * NC (NC = 192) idle
    for (int64_t base = (int64_t)blockIdx.x * SPB; base < total; base += (int64_t)gridDim.x * SPB) {
        const int64_t row = base + q;
        const bool ok = inq && row < total && c < N;
        double common = 0.0;
        bool bad = false;
        const double l = ok ? emission_any<R>(m, o, row, c, &common, &bad) : -__builtin_inf();
        const double wmx = wave_max_dbl(l);
        const int wbad = __any(bad);
        if (inq && (threadIdx.x & 63) == 0) {
            wm[wv] = wmx;
            wb[wv] = wbad;
        }
        __syncthreads();
        double mx = -__builtin_inf();
        int anyb = 0;
        if (inq) {
            for (int k = 0; k < WPS; ++k) {
                mx = fmax(mx, wm[q * WPS + k]);
                anyb |= wb[q * WPS + k];
            }
        }
        __syncthreads();
        if (ok) etab[row * N + c] = (l == -__builtin_inf()) ? (R)0 : fexp_e((R)(l - mx));
        if (inq && row < total && c == 0) mt[row] = anyb ? __builtin_nan("") : mx + common;
    }
}

// largest entry of a non-negative vector spread over the block (every part
// holds the same values; the waves of part 0 publish their maxima)
template <typename R>
__device__ __forceinline__ R blk_max(R v, R *wred, int NC) {
    const R w = wave_max_r(v);
    if (threadIdx.x < (unsigned)NC && (threadIdx.x & 63) == 0) wred[threadIdx.x / 64] = w;
    __syncthreads();
    R mx = wred[0];
    for (int k = 1; k < NC / 64; ++k) mx = fmax(mx, wred[k]);
    return mx;
}

// ---------------------------------------------------------------- 2. forward
template <typename R>
__global__ __launch_bounds__(BT) void k_blk_fwd(StagedModel<R> m, const int64_t *__restrict__ offsets,
                                                const R *__restrict__ etab,
                                                const double *__restrict__ mt, R *__restrict__ alpha,
                                                int32_t *__restrict__ aexp,
                                                double *__restrict__ loglik,
                                                int32_t *__restrict__ status) {
    __shared__ R x[BT];
    __shared__ R psum[4][BT];
    __shared__ R wred[4];
    __shared__ R wsum[4];
    const int N = m.N, NC = blk_nc(N), P = BT / NC, RP = NC / P;
    const int tid = threadIdx.x, c = tid % NC, p = tid / NC;
    const bool live = c < N;
    const int64_t b = blockIdx.x;
    const int64_t off = offsets[b];
    const int T = (int)(offsets[b + 1] - off);
    // t = 0
    R v = live ? m.pi[c] * etab[off * N + c] : (R)0;
    int ex = fexp(blk_max(v, wred, NC));
    v = fldexp(v, -ex);
    int64_t E = ex;
    double logS = mt[off];
    if (p == 0) x[c] = v;
    if (p == 0 && live) alpha[off * N + c] = v;
    if (tid == 0) aexp[off] = ex;
    __syncthreads();
    for (int t = 1; t < T; ++t) {
        const int64_t row = off + t;
        const R e = live ? etab[row * N + c] : (R)0;
        R acc0 = (R)0, acc1 = (R)0;
        const int i0 = p * RP;
        int k = 0;
        for (; k + 1 < RP; k += 2) {
            const int i = i0 + k;
            if (i + 1 < N) {
                acc0 = fma(x[i], live ? m.A[i * N + c] : (R)0, acc0);
                acc1 = fma(x[i + 1], live ? m.A[(i + 1) * N + c] : (R)0, acc1);
            } else if (i < N) {
                acc0 = fma(x[i], live ? m.A[i * N + c] : (R)0, acc0);
            }
        }
        psum[p][c] = acc0 + acc1;
        __syncthreads();
        R s = psum[0][c];
        for (int q = 1; q < P; ++q) s += psum[q][c];
        v = s * e;
        ex = fexp(blk_max(v, wred, NC));
        v = fldexp(v, -ex);
        if (p == 0) x[c] = v;
        if (p == 0 && live) alpha[row * N + c] = v;
        if (tid == 0) aexp[row] = ex;
        E += ex;
        logS += mt[row];
        __syncthreads();
    }
    // log P(y): sum of the last normalised alpha (part 0 waves)
    R tot = wave_sum_r((p == 0) ? v : (R)0);
    if (tid < NC && (tid & 63) == 0) wsum[tid / 64] = tot;
    __syncthreads();
    if (tid == 0) {
        R z = wsum[0];
        for (int q = 1; q < NC / 64; ++q) z += wsum[q];
        double ll;
        int st;
        if (*m.perr) {
            ll = __builtin_nan("");
            st = 4;
        } else if (isnan(logS)) {
            ll = __builtin_nan("");
            st = 2;
        } else if (!(z > (R)0) || isinf(logS)) {
            ll = -__builtin_inf();
            st = 1;
        } else {
            ll = logS + (double)E * 0.69314718055994530942 + log((double)z);
            st = 0;
        }
        loglik[b] = ll;
        status[b] = st;
    }
}

// ---------------------------------------------------------------- 3. backward
template <typename R>
__global__ __launch_bounds__(BT) void k_blk_bwd(StagedModel<R> m, const int64_t *__restrict__ offsets,
                                                R *__restrict__ etab, const R *__restrict__ alpha,
                                                const int32_t *__restrict__ aexp,
                                                const int32_t *__restrict__ status,
                                                R *__restrict__ gamma) {
    __shared__ R xw[BT];
    __shared__ R psum[4][BT];
    __shared__ R wred[4];
    __shared__ R wsum[4];
    const int N = m.N, NC = blk_nc(N), P = BT / NC, RP = NC / P;
    const int tid = threadIdx.x, r = tid % NC, p = tid / NC;
    const bool live = r < N;
    const int64_t b = blockIdx.x;
    const int64_t off = offsets[b];
    const int T = (int)(offsets[b + 1] - off);
    const bool use = status[b] == 0;
    R bt = live ? (R)1 : (R)0;   // beta^_t of state r (identical in every part)
    for (int t = T - 1; t >= 0; --t) {
        const int64_t row = off + t;
        const R a = live ? alpha[row * N + r] : (R)0;
        const R e = live ? etab[row * N + r] : (R)0;
        const R h = a * bt;
        const R w = e * bt;
        if (p == 0) xw[r] = w;
        const R hs = wave_sum_r((p == 0) ? h : (R)0);
        if (tid < NC && (tid & 63) == 0) wsum[tid / 64] = hs;
        __syncthreads();
        R Z = wsum[0];
        for (int q = 1; q < NC / 64; ++q) Z += wsum[q];
        const R rz = (R)1 / Z;
        if (p == 0 && live) {
            gamma[row * N + r] = use ? h * rz : (R)0;
            etab[row * N + r] = (use && t > 0) ? fldexp(w * rz, -aexp[row]) : (R)0;
        }
        if (t == 0) break;
        R acc0 = (R)0, acc1 = (R)0;
        const int k0 = p * RP;
        int k = 0;
        for (; k + 1 < RP; k += 2) {
            const int kk = k0 + k;
            if (kk + 1 < N) {
                acc0 = fma(xw[kk], live ? m.AT[kk * N + r] : (R)0, acc0);
                acc1 = fma(xw[kk + 1], live ? m.AT[(kk + 1) * N + r] : (R)0, acc1);
            } else if (kk < N) {
                acc0 = fma(xw[kk], live ? m.AT[kk * N + r] : (R)0, acc0);
            }
        }
        psum[p][r] = acc0 + acc1;
        __syncthreads();
        R s = psum[0][r];
        for (int q = 1; q < P; ++q) s += psum[q][r];
        const int ex = fexp(blk_max(s, wred, NC));
        bt = fldexp(s, -ex);
    }
}

// ---------------------------------------------------------------- 5. statistics
// gamma_1 summed over the sequences with status 0
template <typename R>
__global__ __launch_bounds__(BT) void k_blk_gamma1(int N, int64_t nseq, const int64_t *offsets,
                                                   const int32_t *status, const R *gamma,
                                                   double *g1) {
    const int c = blockIdx.x * BT + threadIdx.x;
    if (c >= N) return;
    double s = 0.0;
    for (int64_t b = 0; b < nseq; ++b)
        if (status[b] == 0) s += (double)gamma[offsets[b] * N + c];
    g1[c] = s;
}

// gamma-weighted family sums.  Thread (state c, dimension d); the blocks
// of grid row y cover disjoint states over the tile of BLK_TS steps starting
// at y * BLK_TS and fill partial row y = [- | sum gamma (N) | family (N x K)]
// (each entry written once).  Rows of sequences with status != 0 are zero in
// gamma and add nothing.
template <typename R>
__global__ __launch_bounds__(BT) void k_blk_gstats(StagedModel<R> m, ObsRef o, int64_t total,
                                                   const R *__restrict__ gamma,
                                                   double *__restrict__ partial, int64_t S2) {
    const int N = m.N, D = m.D, fam = m.family;
    const int DD = (fam == HMM_DIAG_GAUSSIAN) ? D : 1;
    const int spb = BT / DD;                   // states per block
    const int c = blockIdx.x * spb + threadIdx.x / DD;
    const int d = threadIdx.x % DD;
    if ((int)threadIdx.x >= spb * DD || c >= N) return;
    const int64_t t0 = (int64_t)blockIdx.y * BLK_TS;
    const int64_t t1 = t0 + BLK_TS < total ? t0 + BLK_TS : total;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, g = 0.0;
    const StateConsts<R> k = load_consts(m.ep, c, true);
    const double mu = fam == HMM_DIAG_GAUSSIAN ? (double)m.mv[(size_t)c * D + d] : (double)k.c0;
#pragma unroll 8
    for (int64_t t = t0; t < t1; ++t) {
        const double gm = (double)gamma[t * N + c];
        const double y = (double)load_obs<R>(o, fam == HMM_DIAG_GAUSSIAN ? t * D + d : t);
        if (!(gm > 0.0)) continue;
        g += gm;
        if (fam == HMM_GAUSSIAN || fam == HMM_DIAG_GAUSSIAN) {
            const double dv = y - mu;
            a0 += gm * dv;
            a1 += gm * dv * dv;
        } else if (fam == HMM_GAMMA) {
            a0 += gm * y;
            a1 += gm * log(y);
            a2 += gm * y * y;
        } else if (fam == HMM_STUDENT_T) {
            const double dv = y - mu;
            const double u = (double)k.c4 / (1.0 + (double)k.c1 * dv * dv);
            a0 += gm * u;
            a1 += gm * u * dv;
            a2 += gm * u * dv * dv;
            a3 += gm * (log(u) - u);
        } else if (fam == HMM_POISSON) {
            a0 += gm * y;
        }
    }
    double *row = partial + (int64_t)blockIdx.y * S2;
    const int K = family_k_hd(fam, D);
    if (d == 0) row[1 + c] = g;
    double *f = row + 1 + N + (int64_t)c * K;
    switch (fam) {
    case HMM_GAUSSIAN: f[0] = a0; f[1] = a1; break;
    case HMM_GAMMA: f[0] = a0; f[1] = a1; f[2] = a2; break;
    case HMM_STUDENT_T: f[0] = a0; f[1] = a1; f[2] = a2; f[3] = a3; break;
    case HMM_POISSON: f[0] = a0; break;
    case HMM_DIAG_GAUSSIAN: f[d] = a0; f[D + d] = a1; break;
    default: break;
    }
}

__global__ __launch_bounds__(BT) void k_blk_zero(double *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT)
        p[i] = 0.0;
}

// stats = [sum logL | gamma_1 | xi (sum of GEMM chunks, column-major, times a_ij)
//          | sum gamma | family]
template <typename R>
__global__ __launch_bounds__(BT) void k_blk_assemble(StagedModel<R> m, const R *xi_chunks,
                                                     int nch, const double *g1,
                                                     const double *compact, int64_t S,
                                                     double *stats) {
    const int N = m.N;
    const int64_t NN = (int64_t)N * N;
    for (int64_t s = (int64_t)blockIdx.x * BT + threadIdx.x; s < S; s += (int64_t)gridDim.x * BT) {
        double v;
        if (s == 0) {
            v = compact[0];
        } else if (s <= N) {
            v = g1[s - 1];
        } else if (s <= N + NN) {
            const int64_t k = s - 1 - N;
            const int i = (int)(k / N), j = (int)(k % N);
            double acc = 0.0;
            for (int q = 0; q < nch; ++q) acc += (double)xi_chunks[(int64_t)q * NN + (int64_t)j * N + i];
            v = acc * (double)m.A[k];
        } else {
            v = compact[s - NN - N];   // [sum gamma | family] follow sum logL in the compact vector
        }
        stats[s] = v;
    }
}

// ---------------------------------------------------------------- host side
static rocblas_handle blas_handle() {
    thread_local rocblas_handle h = nullptr;
    if (!h && rocblas_create_handle(&h) != rocblas_status_success) h = nullptr;
    return h;
}

static hmm_status xi_gemm(const float *alpha, const float *wp, int N, int64_t K, int kc, float *C,
                          int nch, hipStream_t s) {
    rocblas_handle h = blas_handle();
    if (!h || rocblas_set_stream(h, s) != rocblas_status_success) return HMM_ERR_DEVICE;
    const float one = 1.0f, zero = 0.0f;
    const int64_t full = K / kc, rem = K - full * kc;
    if (full > 0 &&
        rocblas_sgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_transpose, N, N, kc,
                                      &one, alpha, N, (rocblas_stride)kc * N, wp, N,
                                      (rocblas_stride)kc * N, &zero, C, N, (rocblas_stride)N * N,
                                      (rocblas_int)full) != rocblas_status_success)
        return HMM_ERR_DEVICE;
    if (rem > 0 &&
        rocblas_sgemm(h, rocblas_operation_none, rocblas_operation_transpose, N, N, (rocblas_int)rem,
                      &one, alpha + full * kc * N, N, wp + full * kc * N, N, &zero,
                      C + full * (int64_t)N * N, N) != rocblas_status_success)
        return HMM_ERR_DEVICE;
    (void)nch;
    return HMM_OK;
}

static hmm_status xi_gemm(const double *alpha, const double *wp, int N, int64_t K, int, double *C,
                          int, hipStream_t s) {
    rocblas_handle h = blas_handle();
    if (!h || rocblas_set_stream(h, s) != rocblas_status_success) return HMM_ERR_DEVICE;
    const double one = 1.0, zero = 0.0;
    if (rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, N, N, (rocblas_int)K,
                      &one, alpha, N, wp, N, &zero, C, N) != rocblas_status_success)
        return HMM_ERR_DEVICE;
    return HMM_OK;
}

int blk_xi_chunks(bool f64, int64_t total) {
    if (f64 || total <= 1) return 1;
    const int64_t K = total - 1;
    return (int)((K + BLK_KC - 1) / BLK_KC);
}

int blk_gstats_tiles(int64_t total) { return (int)((total + BLK_TS - 1) / BLK_TS); }

template <typename R>
hmm_status run_block(const StagedModel<R> &m, const ObsDesc &o, const BlockBuffers &bb,
                     double *loglik, int32_t *status, void *gamma_out, double *stats, int64_t S,
                     hipStream_t s) {
    const int N = m.N;
    if (o.nseq == 0) return HMM_OK;
    if (N > BT) return HMM_ERR_UNSUPPORTED;
    R *etab = (R *)bb.etab, *alpha = (R *)bb.alpha;
    R *gamma = gamma_out ? (R *)gamma_out : (R *)bb.gamma;
    const ObsRef obs{o.obs, o.obs_f64};
    const int64_t total = bb.total;
    {
        ProfScope ps("block_emit", s);
        const int spb = BT / blk_nc(N);
        const int64_t nb = (total + spb - 1) / spb;
        hipLaunchKernelGGL(k_blk_emit<R>, dim3((unsigned)(nb < 8192 ? nb : 8192)), dim3(BT), 0, s, m,
                           obs, total, etab, bb.mt);
    }
    {
        ProfScope ps("block_fwd", s);
        hipLaunchKernelGGL(k_blk_fwd<R>, dim3((unsigned)o.nseq), dim3(BT), 0, s, m, o.offsets,
                           (const R *)etab, (const double *)bb.mt, alpha, bb.aexp, loglik, status);
    }
    if (!gamma_out && !stats) return HMM_OK;
    {
        ProfScope ps("block_bwd", s);
        hipLaunchKernelGGL(k_blk_bwd<R>, dim3((unsigned)o.nseq), dim3(BT), 0, s, m, o.offsets, etab,
                           (const R *)alpha, (const int32_t *)bb.aexp, (const int32_t *)status,
                           gamma);
    }
    if (!stats) return HMM_OK;
    if (m.family == HMM_FULL_GAUSSIAN) return HMM_ERR_UNSUPPORTED;
    const int K = family_k_hd(m.family, m.D);
    const int64_t S2 = 1 + N + (int64_t)N * K;
    const int ntile = blk_gstats_tiles(total);
    const int DD = m.family == HMM_DIAG_GAUSSIAN ? m.D : 1;
    const int spb = BT / DD;
    const int ncb = (N + spb - 1) / spb;
    {
        ProfScope ps("block_gstats", s);
        if (m.family == HMM_TABLE) {
            const int64_t nz = (int64_t)ntile * S2;
            hipLaunchKernelGGL(k_blk_zero,
                               dim3((unsigned)((nz + BT - 1) / BT < 4096 ? (nz + BT - 1) / BT : 4096)),
                               dim3(BT), 0, s, bb.partial, nz);
        }
        hipLaunchKernelGGL(k_blk_gstats<R>, dim3((unsigned)ncb, (unsigned)ntile), dim3(BT), 0, s, m,
                           obs, total, (const R *)gamma, bb.partial, S2);
        hipLaunchKernelGGL(k_blk_gamma1<R>, dim3((unsigned)((N + BT - 1) / BT)), dim3(BT), 0, s, N,
                           o.nseq, o.offsets, (const int32_t *)status, (const R *)gamma, bb.g1);
    }
    const int nparts = ntile;
    // sum gamma and family sums into the compact vector (entry 0: sum logL)
    launch_reduce_stats(bb.partial, nparts, S2, loglik, status, o.nseq, bb.compact, bb.red, s);
    const int nch = blk_xi_chunks(sizeof(R) == 8, total);
    if (total > 1) {
        ProfScope ps("block_xi_gemm", s);
        hmm_status st = xi_gemm(alpha, etab + N, N, total - 1, BLK_KC, (R *)bb.xi, nch, s);
        if (st != HMM_OK) return st;
    } else {
        hipLaunchKernelGGL(k_blk_zero, dim3(1), dim3(BT), 0, s, (double *)bb.xi,
                           (int64_t)((size_t)N * N * sizeof(R) / 8 + 1));
    }
    {
        ProfScope ps("block_assemble", s);
        hipLaunchKernelGGL(k_blk_assemble<R>, dim3((unsigned)((S + BT - 1) / BT < 1024 ? (S + BT - 1) / BT : 1024)),
                           dim3(BT), 0, s, m, (const R *)bb.xi, nch, (const double *)bb.g1,
                           (const double *)bb.compact, S, stats);
    }
    return HMM_OK;
}

template hmm_status run_block<float>(const StagedModel<float> &, const ObsDesc &,
                                     const BlockBuffers &, double *, int32_t *, void *, double *,
                                     int64_t, hipStream_t);
template hmm_status run_block<double>(const StagedModel<double> &, const ObsDesc &,
                                      const BlockBuffers &, double *, int32_t *, void *, double *,
                                      int64_t, hipStream_t);

}  // namespace hmmk
