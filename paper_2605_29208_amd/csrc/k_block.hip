// k_block.hip -- batched forward-backward E-step for large state counts
// (N <= 256) and for the multivariate families, one workgroup per sequence.
//
//   1. emission pass (all steps in parallel): e_t(j) = exp(log b_j(y_t) - m_t)
//      with m_t = max_j log b_j(y_t), and m_t plus the state-independent part
//      in FP64;
//   2. forward sweep (section 3.1 recursion, normalised): alpha^_t = (alpha^_{t-1} A) o e_t
//      scaled by 2^-x_t; every alpha^_t row and x_t are kept, with
//      log P(y) = sum_t m_t + ln2 sum_t x_t + log sum_j alpha^_{T-1}(j);
//   3. backward sweep: beta^_{t-1} = A (e_t o beta^_t) rescaled the same way,
//      and at each step the posterior gamma_t = alpha^_t o beta^_t / Z_t
//      (Z_t = sum_j alpha^_t(j) beta^_t(j)) and
//        w'_t = e_t o beta^_t * 2^-x_t / Z_t,
//      which makes xi_t(i,j) = alpha^_{t-1}(i) a_ij w'_t(j) (the normaliser of
//      xi_t, sum_ij alpha^_{t-1}(i) a_ij e_t(j) beta^_t(j), equals 2^x_t Z_t);
//      w'_t overwrites e_t in place;
//   4. sum_t xi_t = (sum_t alpha^_{t-1}^T w'_t) o A: a dense contraction over
//      all steps of all sequences on the matrix cores (k_xi.hip; rows of the
//      first step of a sequence have w' = 0, so pairing row r of alpha^ with
//      row r + 1 of w' across the whole batch is exact);
//   5. gamma-weighted family sums (all steps in parallel, one thread per
//      (state, dimension)), gamma_1, and the assembly of the statistics.
//
// The vector-ALU sweeps of steps 2-3 are in k_sweep.hip and the scaled
// bf16/fp16 matrix-core sweeps in k_grp.hip; this file holds the emission and
// family-sum kernels and the host side of the path.

#include "dev_common.hpp"
#include "hmm_internal.hpp"

namespace hmmk {

constexpr int BT = 256;   // threads of the sweep and emission blocks

__device__ __forceinline__ double wave_max_dbl(double v) {
    return wave_all(v, [](double x, double y) { return fmax(x, y); });
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

// Diagonal-Gaussian emissions: a tile of ES steps has its observations
// staged in LDS; thread j (state j, constants in registers) evaluates
// log b_j for every step of the tile into LDS; then each wave takes steps,
// forms the per-step maximum and writes the factors (coalesced rows).
// RAW: the rows receive log b itself (NaN for a non-finite observation) and
// mt is not written -- the log-emission table of the wave route.
// Blocks take tiles in turn (grid-stride), so each thread loads its state's
// constants once for many tiles; double precision uses half-size tiles so
// that four blocks fit a compute unit's LDS.
template <typename R>
constexpr int emit_es() { return sizeof(R) == 8 ? 16 : 32; }
constexpr int EMIT_BLOCKS = 2048;
template <typename R, int DM, bool RAW>
__global__ __launch_bounds__(BT) void k_blk_emit_diag(StagedModel<R> m, ObsRef o, int64_t total,
                                                      R *__restrict__ etab, double *__restrict__ mt) {
    constexpr int ES = emit_es<R>();
    __shared__ R ysh[ES][DM];
    __shared__ R lsh[ES][BT + 1];
    __shared__ int bsh[ES];
    const int N = m.N, D = m.D, j = threadIdx.x, lane = j & 63, wv = j >> 6;
    const bool live = j < N;
    R mu[DM], wq[DM];
#pragma unroll
    for (int d = 0; d < DM; ++d) {
        mu[d] = (live && d < D) ? m.mv[(size_t)j * D + d] : (R)0;
        wq[d] = (live && d < D) ? m.mv[(size_t)N * D + (size_t)j * D + d] : (R)0;
    }
    const R c0 = live ? m.ep[j * EP_STRIDE] : (R)0;
    // FP64 expands w (y - mu)^2 = y (w y - 2 w mu) + w mu^2: two FMA per
    // dimension instead of three operations; the cancellation costs about
    // log10(mu^2 / var) digits, which FP64 affords.  FP32 keeps the centred form.
    constexpr bool EXPD = sizeof(R) == 8;
    R bq[DM];
    R c1 = c0;
#pragma unroll
    for (int d = 0; d < DM; ++d) {
        bq[d] = (R)-2 * wq[d] * mu[d];
        if constexpr (EXPD) c1 = fma(wq[d] * mu[d], mu[d], c1);
    }
    for (int64_t base = (int64_t)blockIdx.x * ES; base < total; base += (int64_t)gridDim.x * ES) {
        const int ns = (int)((total - base) < ES ? (total - base) : ES);
        __syncthreads();
        if (j < ES) bsh[j] = 0;
        __syncthreads();
        for (int k = j; k < ns * D; k += BT) {
            const int sidx = k / D, d = k % D;
            const R y = load_obs<R>(o, (base + sidx) * D + d);
            ysh[sidx][d] = y;
            if (!isfinite(y)) bsh[sidx] = 1;
        }
        __syncthreads();
        if (live) {
            for (int sidx = 0; sidx < ns; ++sidx) {
                R acc = EXPD ? c1 : c0;
#pragma unroll
                for (int d = 0; d < DM; ++d) {
                    if (d < D) {
                        const R y = ysh[sidx][d];
                        if constexpr (EXPD) {
                            acc = fma(y, fma(wq[d], y, bq[d]), acc);
                        } else {
                            const R dv = y - mu[d];
                            acc = fma(wq[d], dv * dv, acc);
                        }
                    }
                }
                lsh[sidx][j] = acc;
            }
        }
        __syncthreads();
        for (int sidx = wv; sidx < ns; sidx += BT / 64) {
            R l[4];
            R mx = neg_inf<R>();
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int jj = lane + 64 * k;
                l[k] = jj < N ? lsh[sidx][jj] : neg_inf<R>();
                mx = fmax(mx, l[k]);
            }
            mx = wave_max_r(mx);
            const int64_t row = base + sidx;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int jj = lane + 64 * k;
                if constexpr (RAW) {
                    if (jj < N) etab[row * N + jj] = bsh[sidx] ? (R)__builtin_nan("") : l[k];
                } else {
                    if (jj < N) etab[row * N + jj] = (l[k] == neg_inf<R>()) ? (R)0 : fexp_e(l[k] - mx);
                }
            }
            if constexpr (!RAW)
                if (lane == 0) mt[row] = bsh[sidx] ? __builtin_nan("") : (double)mx;
        }
    }
}

// Full-covariance Gaussian emissions, one lane per step: the lane keeps
// its observation in registers and, for each state j in turn (uniform across
// the wave), forms z = L_j^{-1} (y - mu_j) by the lower-triangular product
// and log b_j(y) = c_j - |z|^2 / 2 (c_j = -log det L_j - D log(2 pi) / 2).
// L_j^{-1}, mu_j and c_j are read through the scalar unit (uniform addresses,
// no aliasing stores), so the D(D+1)/2 multiply-adds per state take their
// matrix operand from scalar registers.  The log-densities go to the row
// first; a second pass over the row, which stays in cache, subtracts the
// row maximum and exponentiates (RAW: the row keeps log b, NaN for a
// non-finite observation, and mt is not written).
template <typename R, int DM, bool RAW, bool EXACT>
__global__ __launch_bounds__(64) void k_blk_emit_full(int N, int D_, ObsRef o, int64_t total,
                                                      const R *__restrict__ mu,
                                                      const R *__restrict__ Linv,
                                                      const R *__restrict__ ep,
                                                      R *__restrict__ etab, double *__restrict__ mt) {
    // EXACT: D == DM at compile time (contiguous, batched scalar loads)
    const int D = EXACT ? DM : D_;
    const int64_t row = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const bool ok = row < total;
    R y[DM];
    bool bad = false;
#pragma unroll
    for (int d = 0; d < DM; ++d) {
        y[d] = (ok && d < D) ? load_obs<R>(o, row * D + d) : (R)0;
        bad |= !isfinite(y[d]);
    }
    R *out = etab + (ok ? row : 0) * N;
    R mx = neg_inf<R>();
    for (int j = 0; j < N; ++j) {
        const R *W = Linv + (size_t)j * D * D;
        const R *mj = mu + (size_t)j * D;
        // scalar loads at clamped indices (unconditional, so they are batched);
        // entries past D meet dv = 0 or are left out of q
        R dv[DM];
#pragma unroll
        for (int d = 0; d < DM; ++d) {
            const R mjd = mj[EXACT ? d : (d < D ? d : D - 1)];
            dv[d] = d < D ? y[d] - mjd : (R)0;
        }
        R q = (R)0;
#pragma unroll
        for (int r = 0; r < DM; ++r) {
            const R *Wr = W + (size_t)(EXACT ? r : (r < D ? r : D - 1)) * D;
            R acc = Wr[0] * dv[0];
#pragma unroll
            for (int c = 1; c <= r; ++c) acc = fma(Wr[EXACT ? c : (c < D ? c : D - 1)], dv[c], acc);
            q = r < D ? fma(acc, acc, q) : q;
        }
        const R l = ep[j * EP_STRIDE] - (R)0.5 * q;
        mx = fmax(mx, l);
        if (ok) out[j] = l;
    }
    if (!ok) return;
    if constexpr (RAW) {
        if (bad)
            for (int j = 0; j < N; ++j) out[j] = (R)__builtin_nan("");
        return;
    }
    for (int j = 0; j < N; ++j) {
        const R l = out[j];
        out[j] = (l == neg_inf<R>()) ? (R)0 : fexp_e(l - mx);
    }
    mt[row] = bad ? __builtin_nan("") : (double)mx;
}

// ---------------------------------------------------------------- 5. statistics
// gamma_1 summed over the sequences with status 0
template <typename R>
__global__ __launch_bounds__(BT) void k_blk_gamma1(int N, int64_t nseq, const int64_t *offsets,
                                                   const int32_t *status, const R *gamma,
                                                   double *g1) {
    __shared__ int64_t osh[BT];
    __shared__ int32_t ssh[BT];
    const int tid = threadIdx.x, c = blockIdx.x * BT + tid;
    double s = 0.0;
    // the offsets and statuses of BT sequences staged in LDS in one round,
    // then 32 sequences' loads in flight at clamped indices, added in order
    constexpr int U = 32;
    for (int64_t b0 = 0; b0 < nseq; b0 += BT) {
        const int nb = (int)(nseq - b0 < BT ? nseq - b0 : BT);
        __syncthreads();
        if (tid < nb) {
            osh[tid] = offsets[b0 + tid];
            ssh[tid] = status[b0 + tid];
        }
        __syncthreads();
        if (c < N) {
            for (int u0 = 0; u0 < nb; u0 += U) {
                R g[U];
#pragma unroll
                for (int u = 0; u < U; ++u) g[u] = gamma[osh[u0 + u < nb ? u0 + u : nb - 1] * N + c];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (u0 + u < nb && ssh[u0 + u] == 0) s += (double)g[u];
            }
        }
    }
    if (c < N) g1[c] = s;
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
        const double g0 = (double)gamma[t * N + c];
        const double gm = g0 > 0.0 ? g0 : 0.0;
        const double yr = (double)load_obs<R>(o, fam == HMM_DIAG_GAUSSIAN ? t * D + d : t);
        // a zero weight adds nothing; keep y inside every family's domain there
        const double y = gm > 0.0 ? yr : 1.0;
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

// Same sums with one thread per state (N <= 256) and all DM dimensions of a
// diagonal state in its registers: gamma rows are read whole (coalesced) and
// the observation row is the same for every thread (uniform loads).  Blocks
// take tiles of BLK_TS steps in turn and write one partial row each.
template <typename R, int FAM, int DM>
__global__ __launch_bounds__(BT) void k_blk_gstats_row(StagedModel<R> m, ObsRef o, int64_t total,
                                                       const R *__restrict__ gamma,
                                                       double *__restrict__ partial, int64_t S2) {
    const int N = m.N, D = m.D, c = threadIdx.x;
    const bool live = c < N;
    constexpr int NA = FAM == HMM_DIAG_GAUSSIAN ? 2 * DM : 4;
    double acc[NA], g = 0.0;
#pragma unroll
    for (int k = 0; k < NA; ++k) acc[k] = 0.0;
    const StateConsts<R> kc = load_consts(m.ep, live ? c : 0, true);
    R mu[DM];
#pragma unroll
    for (int d = 0; d < DM; ++d)
        mu[d] = (FAM == HMM_DIAG_GAUSSIAN && live && d < D) ? m.mv[(size_t)c * D + d] : (R)0;
    const int ntile = (int)((total + BLK_TS - 1) / BLK_TS);
    for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t t0 = (int64_t)tile * BLK_TS;
        const int64_t t1 = t0 + BLK_TS < total ? t0 + BLK_TS : total;
#pragma unroll 4
        for (int64_t t = t0; t < t1; ++t) {
            const double g0 = live ? (double)gamma[t * N + c] : 0.0;
            const double gm = g0 > 0.0 ? g0 : 0.0;
            g += gm;
            if constexpr (FAM == HMM_DIAG_GAUSSIAN) {
#pragma unroll
                for (int d = 0; d < DM; ++d) {
                    if (d < D) {
                        const double dv = (double)load_obs<R>(o, t * D + d) - (double)mu[d];
                        acc[d] += gm * dv;
                        acc[DM + d] += gm * dv * dv;
                    }
                }
            } else {
                const double yr = (double)load_obs<R>(o, t);
                const double y = gm > 0.0 ? yr : 1.0;   // a zero weight adds nothing
                if constexpr (FAM == HMM_GAUSSIAN) {
                    const double dv = y - (double)kc.c0;
                    acc[0] += gm * dv;
                    acc[1] += gm * dv * dv;
                } else if constexpr (FAM == HMM_GAMMA) {
                    acc[0] += gm * y;
                    acc[1] += gm * log(y);
                    acc[2] += gm * y * y;
                } else if constexpr (FAM == HMM_STUDENT_T) {
                    const double dv = y - (double)kc.c0;
                    const double u = (double)kc.c4 / (1.0 + (double)kc.c1 * dv * dv);
                    acc[0] += gm * u;
                    acc[1] += gm * u * dv;
                    acc[2] += gm * u * dv * dv;
                    acc[3] += gm * (log(u) - u);
                } else if constexpr (FAM == HMM_POISSON) {
                    acc[0] += gm * y;
                }
            }
        }
    }
    if (!live) return;
    double *row = partial + (int64_t)blockIdx.x * S2;
    row[1 + c] = g;
    const int K = family_k_hd(FAM, D);
    double *f = row + 1 + N + (int64_t)c * K;
    if constexpr (FAM == HMM_DIAG_GAUSSIAN) {
#pragma unroll
        for (int d = 0; d < DM; ++d)
            if (d < D) {
                f[d] = acc[d];
                f[D + d] = acc[DM + d];
            }
    } else {
        for (int k = 0; k < K; ++k) f[k] = acc[k];
    }
}

// Diagonal-Gaussian family sums (D <= DM = 16), one thread per state: blocks
// take tiles of BLK_TS steps in turn; each sub-tile of 64 steps has its
// observations staged in LDS (read back as broadcasts) and is summed in R,
// the sub-tile sums are added in FP64.  One partial row per block.
template <typename R, int DM>
__global__ __launch_bounds__(BT) void k_blk_gstats_diag(StagedModel<R> m, ObsRef o, int64_t total,
                                                        const R *__restrict__ gamma,
                                                        double *__restrict__ partial, int64_t S2) {
    // Double precision sums the raw moments sum g y and sum g y^2 (two FMA per
    // state, step and dimension, y^2 staged beside y) and shifts them by mu
    // at the end; the cancellation costs about log10(mu^2 / var) digits,
    // which FP64 affords.  Single precision keeps the centred form.
    constexpr bool RAWM = sizeof(R) == 8;
    constexpr int SB = 64;
    static_assert((SB * DM) % BT == 0, "whole staging rounds");
    __shared__ __align__(16) R ysh[SB][DM];
    __shared__ __align__(16) R y2sh[RAWM ? SB : 1][DM];
    const int N = m.N, D = m.D, c = threadIdx.x;
    const bool live = c < N;
    R mu[DM];
#pragma unroll
    for (int d = 0; d < DM; ++d) mu[d] = (live && d < D) ? m.mv[(size_t)c * D + d] : (R)0;
    double s1[DM], s2[DM], G = 0.0;
#pragma unroll
    for (int d = 0; d < DM; ++d) s1[d] = s2[d] = 0.0;
    const int ntile = (int)((total + BLK_TS - 1) / BLK_TS);
    const int cc = live ? c : N - 1;
    // gamma of 8 steps of a staged block starting at sb (rows clamped into
    // the block's ns steps)
    auto gload = [&](R (&dst)[8], int64_t sbb, int s0b, int nsb) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int st = s0b + u < nsb ? s0b + u : nsb - 1;
            dst[u] = gamma[(sbb + st) * N + cc];
        }
    };
    for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const int64_t t0 = (int64_t)tile * BLK_TS;
        const int64_t t1 = t0 + BLK_TS < total ? t0 + BLK_TS : total;
        // each batch's gamma is requested one batch ahead, so its latency
        // overlaps the previous batch's sums
        R gr[8];
        gload(gr, t0, 0, (int)(t1 - t0 < SB ? t1 - t0 : SB));
        for (int64_t sb = t0; sb < t1; sb += SB) {
            const int ns = (int)(t1 - sb < SB ? t1 - sb : SB);
            __syncthreads();
            // staging and gamma loads at clamped indices (in bounds, no
            // branches), so each batch of loads is in flight together
            {
                R yv[SB * DM / BT];
#pragma unroll
                for (int u = 0; u < SB * DM / BT; ++u) {
                    const int k = c + u * BT, st = k / DM, d = k % DM;
                    const int64_t idx = (sb + (st < ns ? st : ns - 1)) * D + (d < D ? d : D - 1);
                    yv[u] = load_obs<R>(o, idx);
                }
#pragma unroll
                for (int u = 0; u < SB * DM / BT; ++u) {
                    const int k = c + u * BT, st = k / DM, d = k % DM;
                    const R y = (st < ns && d < D) ? yv[u] : (R)0;
                    ysh[st][d] = y;
                    if constexpr (RAWM) y2sh[st][d] = y * y;
                }
            }
            __syncthreads();
            R a1[DM], a2[DM], g = (R)0;
#pragma unroll
            for (int d = 0; d < DM; ++d) a1[d] = a2[d] = (R)0;
            for (int s0 = 0; s0 < SB; s0 += 8) {
                // the next batch: later in this block, else the tile's next block
                R gn[8];
                const bool same = s0 + 8 < SB;
                const int64_t nsb = same ? sb : sb + SB;
                if (nsb < t1) {   // uniform
                    gload(gn, nsb, same ? s0 + 8 : 0, (int)(t1 - nsb < SB ? t1 - nsb : SB));
                } else {
#pragma unroll
                    for (int u = 0; u < 8; ++u) gn[u] = (R)0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const R g0 = (live && s0 + u < ns) ? gr[u] : (R)0;
                    const R gm = g0 > (R)0 ? g0 : (R)0;
                    g += gm;
#pragma unroll
                    for (int d = 0; d < DM; ++d) {
                        if constexpr (RAWM) {
                            a1[d] = fma(gm, ysh[s0 + u][d], a1[d]);
                            a2[d] = fma(gm, y2sh[s0 + u][d], a2[d]);
                        } else {
                            const R dv = ysh[s0 + u][d] - mu[d];
                            const R gd = gm * dv;
                            a1[d] += gd;
                            a2[d] = fma(gd, dv, a2[d]);
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) gr[u] = gn[u];
            }
#pragma unroll
            for (int d = 0; d < DM; ++d) {
                s1[d] += (double)a1[d];
                s2[d] += (double)a2[d];
            }
            G += (double)g;
        }
    }
    if (!live) return;
    double *row = partial + (int64_t)blockIdx.x * S2;
    row[1 + c] = G;
    double *f = row + 1 + N + (int64_t)c * (2 * D);
#pragma unroll
    for (int d = 0; d < DM; ++d)
        if (d < D) {
            if constexpr (RAWM) {
                // sum g (y - mu) and sum g (y - mu)^2 from the raw moments
                const double md = (double)mu[d];
                f[d] = s1[d] - md * G;
                f[D + d] = (s2[d] - 2.0 * md * s1[d]) + md * md * G;
            } else {
                f[d] = s1[d];
                f[D + d] = s2[d];
            }
        }
}

// Full-covariance family sums of one state c over one tile of FULL_TS steps:
// sum gamma, sum gamma (y - mu_c) and the lower triangle of
// sum gamma (y - mu_c)(y - mu_c)^T.  Sub-tiles of 64 steps are staged in LDS
// (centred observations and gamma); thread t owns 2 x 2 blocks of the lower
// triangle (block index t, t + BT, ...), reading two rows and two columns per
// step for four products.  Sums run in R over a sub-tile and in FP64 across
// sub-tiles.
template <typename R, int DM>
__global__ __launch_bounds__(BT) void k_blk_gstats_full2(int N, int D, ObsRef o, int64_t total,
                                                         const R *__restrict__ mu,
                                                         const R *__restrict__ gamma,
                                                         double *__restrict__ partial, int64_t S2) {
    constexpr int SB = 64;                       // steps per sub-tile
    constexpr int HB = DM / 2;                   // 2 x 2 blocks per row of blocks
    constexpr int NB = HB * (HB + 1) / 2;        // lower-triangle blocks
    constexpr int BPT = (NB + BT - 1) / BT;      // blocks per thread
    __shared__ R vs[SB][DM + 1];
    __shared__ R gs[SB];
    const int c = blockIdx.x, tid = threadIdx.x;
    const int K = D + D * (D + 1) / 2;
    const int64_t t0 = (int64_t)blockIdx.y * FULL_TS;
    const int64_t t1 = t0 + FULL_TS < total ? t0 + FULL_TS : total;
    int br[BPT], bc[BPT];
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        int b = tid + u * BT, r = 0;
        if (b >= NB) b = -1;
        if (b >= 0) {   // block b = r (r + 1) / 2 + k of the block triangle
            while ((r + 1) * (r + 2) / 2 <= b) ++r;
        }
        br[u] = b >= 0 ? r : -1;
        bc[u] = b >= 0 ? b - r * (r + 1) / 2 : 0;
    }
    double S[BPT][4], F = 0.0, G = 0.0;
#pragma unroll
    for (int u = 0; u < BPT; ++u) S[u][0] = S[u][1] = S[u][2] = S[u][3] = 0.0;
    for (int64_t sb = t0; sb < t1; sb += SB) {
        const int ns = (int)(t1 - sb < SB ? t1 - sb : SB);
        __syncthreads();
        for (int k = tid; k < SB * DM; k += BT) {
            const int st = k / DM, d = k % DM;
            R v = (R)0;
            if (st < ns && d < D) v = load_obs<R>(o, (sb + st) * D + d) - mu[(size_t)c * D + d];
            vs[st][d] = v;
        }
        if (tid < SB) gs[tid] = tid < ns ? gamma[(sb + tid) * N + c] : (R)0;
        __syncthreads();
        R a[BPT][4], f = (R)0, g = (R)0;
#pragma unroll
        for (int u = 0; u < BPT; ++u) a[u][0] = a[u][1] = a[u][2] = a[u][3] = (R)0;
        for (int st = 0; st < SB; ++st) {
            const R gm = gs[st];
#pragma unroll
            for (int u = 0; u < BPT; ++u) {
                if (br[u] >= 0) {
                    const int r0 = 2 * br[u], c0 = 2 * bc[u];
                    const R x0 = gm * vs[st][r0], x1 = gm * vs[st][r0 + 1];
                    const R w0 = vs[st][c0], w1 = vs[st][c0 + 1];
                    a[u][0] = fma(x0, w0, a[u][0]);
                    a[u][1] = fma(x0, w1, a[u][1]);
                    a[u][2] = fma(x1, w0, a[u][2]);
                    a[u][3] = fma(x1, w1, a[u][3]);
                }
            }
            if (tid < D) f = fma(gm, vs[st][tid], f);
            g += gm;
        }
#pragma unroll
        for (int u = 0; u < BPT; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) S[u][e] += (double)a[u][e];
        F += (double)f;
        G += (double)g;
    }
    double *row = partial + (int64_t)blockIdx.y * S2 + 1 + N + (int64_t)c * K;
    if (tid == 0) partial[(int64_t)blockIdx.y * S2 + 1 + c] = G;
    if (tid < D) row[tid] = F;
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        if (br[u] < 0) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = 2 * br[u] + (e >> 1), k = 2 * bc[u] + (e & 1);
            if (r < D && k <= r) row[D + r * (r + 1) / 2 + k] = S[u][e];
        }
    }
}

__global__ __launch_bounds__(BT) void k_blk_zero(double *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT)
        p[i] = 0.0;
}

// stats = [sum logL | gamma_1 | xi (the contraction times a_ij) | sum gamma | family]
template <typename R>
__global__ __launch_bounds__(BT) void k_blk_assemble(StagedModel<R> m, const double *xisum,
                                                     const double *g1, const double *compact,
                                                     int64_t S, double *stats) {
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
            v = xisum[k] * (double)m.A[k];
        } else {
            v = compact[s - NN - N];   // [sum gamma | family] follow sum logL in the compact vector
        }
        stats[s] = v;
    }
}

// ---------------------------------------------------------------- host side
int blk_gstats_tiles(int64_t total, int family) {
    const int64_t ts = family == HMM_FULL_GAUSSIAN ? FULL_TS : BLK_TS;
    return (int)((total + ts - 1) / ts);
}

// The vector-ALU sweeps (FP32/FP64, 64 < N <= 256) are in k_sweep.hip; the
// scaled low-precision options (any N <= 256) are in k_grp.hip.
template <typename R>
static void launch_blk_sweep(bool fwd, const StagedModel<R> &m, const ObsDesc &o, R *etab,
                             const BlockBuffers &bb, R *alpha, double *loglik, int32_t *status,
                             R *gamma, hipStream_t s) {
    if constexpr (sizeof(R) == 4) {
        if (bb.mfma == 1 || bb.mfma == 2)
            return launch_grp_sweep(fwd, bb.mfma == 1, m, o.offsets, o.nseq, etab, bb.mt, alpha,
                                    bb.aexp, loglik, status, gamma, s);
    }
    // the planner sends N <= 64 to the wave path unless a scaled option is asked for
    launch_sw_sweep<R>(fwd, m, o.offsets, o.nseq, etab, bb.mt, alpha, bb.aexp, loglik, status,
                       gamma, s);
}

// Full-covariance family sums in single precision for D <= 32 on the matrix
// cores: for state c the second moment sum_t gamma_t d_t d_t^T (d = y - mu_c)
// is the product (diag(gamma) V)^T V over the tile's centred observations V,
// taken two steps per v_mfma_f32_32x32x2_f32 (lane l holds dimension l % 32
// of step 2q + l / 32 as both operands, the left one scaled by gamma).  One
// wave per (group of FG states, tile of FULL_TS steps): a step's observation
// and the group's gamma values are loaded once and serve the FG states, whose
// products are independent MFMA chains.  The FP32 accumulators are added into
// FP64 every 64 steps.  Result element (i, j) sits in lane j + 32 ((i / 4) %
// 2), register 4 (i / 8) + i % 4.
typedef float floatx16_t __attribute__((ext_vector_type(16)));
constexpr int FG = 2;   // states per wave
template <typename Y>
__global__ __launch_bounds__(64) void k_blk_gstats_full_mfma(int N, int D, const Y *__restrict__ obs,
                                                            int64_t total,
                                                            const float *__restrict__ mu,
                                                            const float *__restrict__ gamma,
                                                            double *__restrict__ partial,
                                                            int64_t S2) {
    const int c0 = blockIdx.x * FG, l = threadIdx.x, i = l & 31, k = l >> 5;
    const int ic = i < D ? i : D - 1;
    const int K = D + D * (D + 1) / 2;
    const int64_t t0 = (int64_t)blockIdx.y * FULL_TS;
    const int64_t t1 = t0 + FULL_TS < total ? t0 + FULL_TS : total;
    int cs[FG];
    float mui[FG];
#pragma unroll
    for (int g = 0; g < FG; ++g) {
        cs[g] = c0 + g < N ? c0 + g : N - 1;
        mui[g] = mu[(size_t)cs[g] * D + ic];
    }
    double S[FG][16], F[FG], G[FG];
#pragma unroll
    for (int g = 0; g < FG; ++g) {
        F[g] = 0.0;
        G[g] = 0.0;
#pragma unroll
        for (int v = 0; v < 16; ++v) S[g][v] = 0.0;
    }
    const Y *ot = obs + t0 * D;
    const float *gt = gamma + t0 * N;
    const int nrow = (int)(t1 - t0);
    for (int64_t base = t0; base < t1; base += 64) {
        floatx16_t acc[FG];
        float f[FG], gs[FG];
#pragma unroll
        for (int g = 0; g < FG; ++g) {
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[g][v] = 0.0f;
            f[g] = 0.0f;
            gs[g] = 0.0f;
        }
        // batches of 8 step pairs: all loads first, at clamped indices (always
        // in bounds, no branches), so they are in flight together
        // rows addressed from the tile's first row in 32-bit offsets (a tile
        // holds at most FULL_TS steps)
        for (int q0 = 0; q0 < 32; q0 += 8) {
            float gr[8][FG], yr[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int tr = (int)(base - t0) + 2 * (q0 + u) + k;
                const int tc = tr < nrow ? tr : nrow - 1;
                yr[u] = (float)ot[tc * D + ic];
#pragma unroll
                for (int g = 0; g < FG; ++g) gr[u][g] = gt[tc * N + cs[g]];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool on = base + 2 * (q0 + u) + k < t1;
#pragma unroll
                for (int g = 0; g < FG; ++g) {
                    const float gm = on ? gr[u][g] : 0.0f;
                    const float dv = (on && i < D) ? yr[u] - mui[g] : 0.0f;
                    const float a = gm * dv;
                    acc[g] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, dv, acc[g], 0, 0, 0);
                    f[g] += a;
                    gs[g] += gm;
                }
            }
        }
#pragma unroll
        for (int g = 0; g < FG; ++g) {
#pragma unroll
            for (int v = 0; v < 16; ++v) S[g][v] += (double)acc[g][v];
            F[g] += (double)f[g];
            G[g] += (double)gs[g];
        }
    }
    double *row = partial + (int64_t)blockIdx.y * S2;
#pragma unroll
    for (int g = 0; g < FG; ++g) {
        const int c = c0 + g;
        // first moments and sum gamma: add the two step parities (lanes l and l ^ 32)
        const double Fo = __shfl_xor(F[g], 32, 64), Go = __shfl_xor(G[g], 32, 64);
        if (c >= N) continue;   // uniform
        if (l == 0) row[1 + c] = G[g] + Go;
        double *fr = row + 1 + N + (int64_t)c * K;
        if (k == 0 && i < D) fr[i] = F[g] + Fo;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int ii = 8 * (v / 4) + 4 * k + (v % 4), jj = i;
            if (ii < D && jj <= ii) fr[D + ii * (ii + 1) / 2 + jj] = S[g][v];
        }
    }
}

// gamma-weighted family sums from gamma rows [total x N] into partial rows
// [- | sum gamma (N) | family (N x K)] of S2 doubles; returns the row count
// (at most blk_gstats_tiles(total, family))
template <typename R>
static int launch_family_sums(const StagedModel<R> &m, const ObsRef &obs, int64_t total,
                              const R *gamma, double *partial, int64_t S2, hipStream_t s) {
    const int N = m.N;
    int nparts = blk_gstats_tiles(total, m.family);
    const bool rowk = !(m.family == HMM_DIAG_GAUSSIAN && m.D > 16);
    if (m.family == HMM_FULL_GAUSSIAN) {
        const dim3 g((unsigned)N, (unsigned)nparts);
        if constexpr (sizeof(R) == 4) {
            if (m.D <= 32) {
                const dim3 gm((unsigned)((N + FG - 1) / FG), (unsigned)nparts);
                if (obs.f64)
                    hipLaunchKernelGGL(k_blk_gstats_full_mfma<double>, gm, dim3(64), 0, s, N, m.D,
                                       (const double *)obs.p, total, (const float *)m.mv,
                                       (const float *)gamma, partial, S2);
                else
                    hipLaunchKernelGGL(k_blk_gstats_full_mfma<float>, gm, dim3(64), 0, s, N, m.D,
                                       (const float *)obs.p, total, (const float *)m.mv,
                                       (const float *)gamma, partial, S2);
                return nparts;
            }
        }
        if (m.D <= 16)
            hipLaunchKernelGGL((k_blk_gstats_full2<R, 16>), g, dim3(BT), 0, s, N, m.D, obs, total,
                               (const R *)m.mv, (const R *)gamma, partial, S2);
        else if (m.D <= 32)
            hipLaunchKernelGGL((k_blk_gstats_full2<R, 32>), g, dim3(BT), 0, s, N, m.D, obs, total,
                               (const R *)m.mv, (const R *)gamma, partial, S2);
        else
            hipLaunchKernelGGL((k_blk_gstats_full2<R, 64>), g, dim3(BT), 0, s, N, m.D, obs, total,
                               (const R *)m.mv, (const R *)gamma, partial, S2);
    } else if (rowk) {
        // one thread per state; blocks take tiles in turn
        nparts = nparts < BLK_GS_BLOCKS ? nparts : BLK_GS_BLOCKS;
        const dim3 g((unsigned)nparts);
        const R *gp = (const R *)gamma;
        switch (m.family) {
        case HMM_GAUSSIAN:
            hipLaunchKernelGGL((k_blk_gstats_row<R, HMM_GAUSSIAN, 1>), g, dim3(BT), 0, s, m, obs, total, gp, partial, S2);
            break;
        case HMM_GAMMA:
            hipLaunchKernelGGL((k_blk_gstats_row<R, HMM_GAMMA, 1>), g, dim3(BT), 0, s, m, obs, total, gp, partial, S2);
            break;
        case HMM_STUDENT_T:
            hipLaunchKernelGGL((k_blk_gstats_row<R, HMM_STUDENT_T, 1>), g, dim3(BT), 0, s, m, obs, total, gp, partial, S2);
            break;
        case HMM_POISSON:
            hipLaunchKernelGGL((k_blk_gstats_row<R, HMM_POISSON, 1>), g, dim3(BT), 0, s, m, obs, total, gp, partial, S2);
            break;
        case HMM_DIAG_GAUSSIAN:
            hipLaunchKernelGGL((k_blk_gstats_diag<R, 16>), g, dim3(BT), 0, s, m, obs, total, gp, partial, S2);
            break;
        default:   // table: sum gamma only
            hipLaunchKernelGGL((k_blk_gstats_row<R, HMM_TABLE, 1>), g, dim3(BT), 0, s, m, obs, total, gp, partial, S2);
            break;
        }
    } else {
        const int DD = m.D;
        const int spb = BT / DD;
        const int ncb = (N + spb - 1) / spb;
        hipLaunchKernelGGL(k_blk_gstats<R>, dim3((unsigned)ncb, (unsigned)nparts), dim3(BT), 0, s, m,
                           obs, total, (const R *)gamma, partial, S2);
    }
    return nparts;
}

// Emission rows of the block path (RAW = false: e_t and m_t) or the raw
// log-density table of the wave route for multivariate families (RAW = true)
template <typename R, bool RAW>
static void launch_blk_emission(const StagedModel<R> &m, const ObsRef &obs, int64_t total, R *etab,
                                double *mt, hipStream_t s) {
    const int N = m.N;
    ProfScope ps("block_emit", s);
    if (m.family == HMM_DIAG_GAUSSIAN && m.D <= 64) {
        const int64_t nb = (total + emit_es<R>() - 1) / emit_es<R>();
        const dim3 g((unsigned)(nb < EMIT_BLOCKS ? nb : EMIT_BLOCKS));
        if (m.D <= 16)
            hipLaunchKernelGGL((k_blk_emit_diag<R, 16, RAW>), g, dim3(BT), 0, s, m, obs, total, etab, mt);
        else
            hipLaunchKernelGGL((k_blk_emit_diag<R, 64, RAW>), g, dim3(BT), 0, s, m, obs, total, etab, mt);
    } else if (m.family == HMM_FULL_GAUSSIAN && m.D <= 64) {
        const dim3 g((unsigned)((total + 63) / 64));
        const R *mu = m.mv, *Li = m.mv + (size_t)N * m.D;
        const R *ep = (const R *)m.ep;
        if (m.D == 16)
            hipLaunchKernelGGL((k_blk_emit_full<R, 16, RAW, true>), g, dim3(64), 0, s, N, m.D, obs, total,
                               mu, Li, ep, etab, mt);
        else if (m.D == 32)
            hipLaunchKernelGGL((k_blk_emit_full<R, 32, RAW, true>), g, dim3(64), 0, s, N, m.D, obs, total,
                               mu, Li, ep, etab, mt);
        else if (m.D == 64)
            hipLaunchKernelGGL((k_blk_emit_full<R, 64, RAW, true>), g, dim3(64), 0, s, N, m.D, obs, total,
                               mu, Li, ep, etab, mt);
        else if (m.D < 16)
            hipLaunchKernelGGL((k_blk_emit_full<R, 16, RAW, false>), g, dim3(64), 0, s, N, m.D, obs, total,
                               mu, Li, ep, etab, mt);
        else if (m.D < 32)
            hipLaunchKernelGGL((k_blk_emit_full<R, 32, RAW, false>), g, dim3(64), 0, s, N, m.D, obs, total,
                               mu, Li, ep, etab, mt);
        else
            hipLaunchKernelGGL((k_blk_emit_full<R, 64, RAW, false>), g, dim3(64), 0, s, N, m.D, obs, total,
                               mu, Li, ep, etab, mt);
    } else if constexpr (!RAW) {
        const int spb = BT / blk_nc(N);
        const int64_t nb = (total + spb - 1) / spb;
        hipLaunchKernelGGL(k_blk_emit<R>, dim3((unsigned)(nb < 8192 ? nb : 8192)), dim3(BT), 0, s, m,
                           obs, total, etab, mt);
    }
}

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
    launch_blk_emission<R, false>(m, obs, total, etab, bb.mt, s);
    {
        ProfScope ps("block_fwd", s);
        launch_blk_sweep<R>(true, m, o, etab, bb, alpha, loglik, status, nullptr, s);
    }
    if (!gamma_out && !stats) return HMM_OK;
    {
        ProfScope ps("block_bwd", s);
        launch_blk_sweep<R>(false, m, o, etab, bb, alpha, loglik, status, gamma, s);
    }
    if (!stats) return HMM_OK;
    const int K = family_k_hd(m.family, m.D);
    const int64_t S2 = 1 + N + (int64_t)N * K;
    int nparts;
    {
        ProfScope ps("block_gstats", s);
        nparts = launch_family_sums<R>(m, obs, total, (const R *)gamma, bb.partial, S2, s);
        hipLaunchKernelGGL(k_blk_gamma1<R>, dim3((unsigned)((N + BT - 1) / BT)), dim3(BT), 0, s, N,
                           o.nseq, o.offsets, (const int32_t *)status, (const R *)gamma, bb.g1);
    }
    // sum gamma and family sums into the compact vector (entry 0: sum logL)
    launch_reduce_stats(bb.partial, nparts, S2, loglik, status, o.nseq, bb.compact, bb.red, s);
    if (total > 1) {
        ProfScope ps("block_xi", s);
        launch_xi_sum<R>(alpha, etab, N, total - 1, (R *)bb.xi, bb.xi_nsl, bb.xisum, s);
    } else {
        hipLaunchKernelGGL(k_blk_zero, dim3(1), dim3(BT), 0, s, bb.xisum, (int64_t)N * N);
    }
    {
        ProfScope ps("block_assemble", s);
        hipLaunchKernelGGL(k_blk_assemble<R>, dim3((unsigned)((S + BT - 1) / BT < 1024 ? (S + BT - 1) / BT : 1024)),
                           dim3(BT), 0, s, m, (const double *)bb.xisum, (const double *)bb.g1,
                           (const double *)bb.compact, S, stats);
    }
    return HMM_OK;
}

template <typename R>
hmm_status run_wave_mv(const StagedModel<R> &m, const ObsDesc &o, const WaveBuffers &wb,
                       const MvBuffers &mb, double *loglik, int32_t *status, void *gamma_out,
                       double *stats, hipStream_t s) {
    if (o.nseq == 0) return HMM_OK;
    const int N = m.N;
    const ObsRef obs{o.obs, o.obs_f64};
    R *lt = (R *)mb.lt;
    launch_blk_emission<R, true>(m, obs, mb.total, lt, nullptr, s);
    StagedModel<R> mtab = m;
    mtab.family = HMM_TABLE;
    const ObsDesc otab{lt, sizeof(R) == 8 ? 1 : 0, o.nseq, o.offsets};
    R *gam = gamma_out ? (R *)gamma_out : (stats ? (R *)mb.gamma : nullptr);
    // the table family's statistics are the prefix [logL | gamma_1 | xi | sum gamma]
    const int64_t Sw = 1 + 2 * (int64_t)N + (int64_t)N * N;
    hmm_status r = run_wave<R>(mtab, otab, wb, loglik, status, gam, stats, Sw, s);
    if (r != HMM_OK || !stats) return r;
    const int K = family_k_hd(m.family, m.D);
    const int64_t S2 = 1 + N + (int64_t)N * K;
    int nparts;
    {
        ProfScope ps("block_gstats", s);
        nparts = launch_family_sums<R>(m, obs, mb.total, gam, mb.partial, S2, s);
    }
    launch_reduce_stats(mb.partial, nparts, S2, loglik, status, o.nseq, mb.compact, mb.red, s);
    hipMemcpyAsync(stats + Sw, mb.compact + 1 + N, (size_t)N * K * sizeof(double),
                   hipMemcpyDeviceToDevice, s);
    return HMM_OK;
}

template hmm_status run_wave_mv<float>(const StagedModel<float> &, const ObsDesc &,
                                       const WaveBuffers &, const MvBuffers &, double *, int32_t *,
                                       void *, double *, hipStream_t);
template hmm_status run_wave_mv<double>(const StagedModel<double> &, const ObsDesc &,
                                        const WaveBuffers &, const MvBuffers &, double *, int32_t *,
                                        void *, double *, hipStream_t);

template hmm_status run_block<float>(const StagedModel<float> &, const ObsDesc &,
                                     const BlockBuffers &, double *, int32_t *, void *, double *,
                                     int64_t, hipStream_t);
template hmm_status run_block<double>(const StagedModel<double> &, const ObsDesc &,
                                      const BlockBuffers &, double *, int32_t *, void *, double *,
                                      int64_t, hipStream_t);

}  // namespace hmmk
