// k_chunk.hip -- batched forward-backward E-step for small state counts
// (N <= 8), exact and time-parallel.
//
// The forward recursion of section 3.2, alpha_t(j) = lse_i[alpha_{t-1}(i) +
// log a_ij] + log b_j(y_t), is carried in linear form on a normalised vector
// with an exact log offset:  alpha_t = (alpha_{t-1} A) o e_t, where
// e_t(j) = exp(log b_j(y_t) - m_t) and m_t = max_j log b_j(y_t); every step
// is rescaled by a power of two (exact) and the exponents and the m_t are
// summed on the side.  Writing M_t = A diag(e_t), a sequence is cut into
// chunks of L steps and each chunk's transfer matrix P_c = prod_{t in c} M_t
// is formed independently (phase 1).  Then, per sequence, the chunk-boundary
// vectors alpha_{end(c)} = alpha_{end(c-1)} P_c and beta_{end(c-1)} = P_c
// beta_{end(c)} follow from a short serial scan over chunks (phase 2).
// Finally every chunk re-runs its own L forward steps from its boundary and
// the backward recursion beta_{t-1} = M_t beta_t down to its start, forming
// gamma_t and xi_t (definitions of section 3.1) and accumulating the
// gamma-weighted statistics of section 4 (phase 3).  The result equals the
// sequential recursion up to rounding; phase 1 costs N^3 per step instead of
// N^2 but has no serial dependency between chunks.
//
// Lanes: a chunk's N x N transfer matrix occupies G*G lanes in phase 1
// (lane = (row i, column j)); in phases 2 and 3 a sequence or chunk occupies
// G lanes (lane = state).  G = 4 (N <= 4) or 8 (N <= 8); the lane exchanges
// inside a group of G lanes are DPP quad permutations and the half-row mirror.
#include <climits>

#include "dev_common.hpp"
#include "hmm_internal.hpp"

namespace hmmk {

struct ChunkGeom {
    int64_t nseq;
    const int64_t *offsets;
    const int *cbase;
    int L;
    int C;
    ObsRef obs;
};

constexpr int LMAX = 64;
constexpr int NEG_EXP = INT_MIN / 4;

// one observation (scalar families) or one log b_j entry (table family)
template <int FAM, typename R>
__device__ __forceinline__ R load_step(const ObsRef &o, int64_t row, int j, int N, bool live) {
    if constexpr (FAM == HMM_TABLE) {
        return live ? load_obs<R>(o, row * N + j) : neg_inf<R>();
    } else {
        return load_obs<R>(o, row);
    }
}

template <int FAM, typename R>
__device__ __forceinline__ Emit<R> emit_step(R v, const StateConsts<R> &k, bool live) {
    if constexpr (FAM == HMM_TABLE) {
        Emit<R> e;
        e.ell = live ? v : neg_inf<R>();
        e.common = 0.0;
        e.bad = live && (isnan(v) || (v > (R)0 && isinf(v)));
        return e;
    } else {
        return emit_scalar<FAM, R>(v, k, live);
    }
}

// ---------------------------------------------------------------- phase 1
template <typename R, int G, int FAM>
__global__ __launch_bounds__(BLOCK) void k_chunk_product(ChunkGeom g, StagedModel<R> m,
                                                         R *__restrict__ Pout,
                                                         int *__restrict__ rexp,
                                                         double *__restrict__ clog) {
    constexpr int GG = G * G;
    constexpr int CPW = 64 / GG;
    constexpr int CPB = (BLOCK / 64) * CPW;
    __shared__ R esh[CPB][LMAX][G];
    __shared__ double msh[CPB][G];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane / GG, li = (lane % GG) / G, lj = lane % G;
    const int slot = wave * CPW + sub;
    const int c = blockIdx.x * CPB + slot;
    const bool valid = c < g.C;
    const int N = m.N;
    int64_t off = 0;
    int ts = 0, nsteps = 0;
    if (valid) {
        int b = find_seq(g.cbase, (int)g.nseq, c);
        off = g.offsets[b];
        int T = (int)(g.offsets[b + 1] - off);
        int t0 = (c - g.cbase[b]) * g.L;
        int t1 = min(t0 + g.L, T);
        ts = max(t0, 1);
        nsteps = max(t1 - ts, 0);
    }
    const int nmax = wave_max_i(nsteps);
    const bool live = lj < N;
    using ET = typename EmitTraits<FAM, R>::T;
    const StateConsts<ET> k = load_consts(consts_ptr<FAM, R>(m), lj, live);

    // emissions of the chunk: row group li takes steps ts + li, ts + li + G, ...
    double msum = 0.0;
    bool bad = false;
    for (int base = 0; base < nmax; base += G) {
        const int tt = base + li;
        const bool act = tt < nsteps;
        R v = act ? load_step<FAM, R>(g.obs, off + ts + tt, lj, N, live) : (R)1;
        Emit<ET> em = emit_step<FAM, ET>((ET)v, k, live);
        ET mx = grp_max<G, ET>(em.ell);
        R e = (em.ell == neg_inf<ET>()) ? (R)0 : fexp_e((R)(em.ell - mx));
        bool gbad = grp_max_i<G>((act && em.bad) ? 1 : 0) > 0;
        if (act) {
            esh[slot][tt][lj] = e;
            msum += (double)mx + em.common;
            bad |= gbad;
        }
    }
    if (lj == 0) msh[slot][li] = bad ? __builtin_nan("") : msum;
    __syncthreads();

    R coef[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
        int i = grp_src(lj, q);
        coef[q] = (live && i < N) ? m.A[i * N + lj] : (R)0;
    }
    R P = (li == lj && live) ? (R)1 : (R)0;
    int r = 0;
    for (int s = 0; s < nmax; ++s) {
        const bool act = s < nsteps;
        R e = esh[slot][act ? s : 0][lj];
        R v = grp_dot<G, R>(P, coef) * e;
        int ex = fexp(grp_max<G, R>(v));
        v = fldexp(v, -ex);
        if (act) {
            P = v;
            r += ex;
        }
    }
    if (valid) {
        Pout[(size_t)c * GG + li * G + lj] = P;
        if (lj == 0) rexp[(size_t)c * G + li] = r;
        if (li == 0 && lj == 0) {
            double t = 0.0;
            for (int q = 0; q < G; ++q) t += msh[slot][q];
            clog[c] = t;
        }
    }
}

// ---------------------------------------------------------------- phase 2
template <typename R, int G, int FAM>
__global__ __launch_bounds__(BLOCK) void k_chunk_scan(ChunkGeom g, StagedModel<R> m,
                                                      const R *__restrict__ P,
                                                      const int *__restrict__ rexp,
                                                      const double *__restrict__ clog,
                                                      R *__restrict__ Fo, R *__restrict__ Go,
                                                      double *__restrict__ loglik,
                                                      int32_t *__restrict__ status) {
    constexpr int GG = G * G, SPW = 64 / G;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane / G, p = lane % G;
    const int64_t b = ((int64_t)blockIdx.x * (BLOCK / 64) + wave) * SPW + sub;
    const bool valid = b < g.nseq;
    const int N = m.N;
    int cb = 0, nch = 0;
    int64_t off = 0;
    if (valid) {
        cb = g.cbase[b];
        nch = g.cbase[b + 1] - cb;
        off = g.offsets[b];
    }
    const int nmax = wave_max_i(nch);
    const bool live = p < N;

    if (blockIdx.y == 0) {
        // forward: alpha_0 = pi o e_0, then alpha_{end(c)} = alpha_{end(c-1)} P_c
        using ET = typename EmitTraits<FAM, R>::T;
        const StateConsts<ET> k = load_consts(consts_ptr<FAM, R>(m), p, live);
        R v0 = valid ? load_step<FAM, R>(g.obs, off, p, N, live) : (R)1;
        Emit<ET> em = emit_step<FAM, ET>((ET)v0, k, live);
        ET mx = grp_max<G, ET>(em.ell);
        R e = (em.ell == neg_inf<ET>()) ? (R)0 : fexp_e((R)(em.ell - mx));
        R f = (live ? m.pi[p] : (R)0) * e;
        double logS = (double)mx + em.common;
        bool bad = grp_max_i<G>(em.bad ? 1 : 0) > 0;
        int ex0 = fexp(grp_max<G, R>(f));
        f = fldexp(f, -ex0);
        int64_t E = ex0;
        for (int s = 0; s < nmax; ++s) {
            const bool act = s < nch;
            const int c = act ? cb + s : 0;
            R coef[G];
#pragma unroll
            for (int q = 0; q < G; ++q)
                coef[q] = act ? P[(size_t)c * GG + grp_src(p, q) * G + p] : (R)0;
            const int rr = act ? rexp[(size_t)c * G + p] : 0;
            const double cl = act ? clog[c] : 0.0;
            const int ce = (f > (R)0) ? fexp(f) + rr : NEG_EXP;
            const int Rm = grp_max_i<G>(ce);
            R w = (f > (R)0) ? fldexp(f, rr - Rm) : (R)0;
            R v = grp_dot<G, R>(w, coef);
            int ev = fexp(grp_max<G, R>(v));
            v = fldexp(v, -ev);
            if (act) {
                f = v;
                E += (int64_t)Rm + ev;
                logS += cl;
                if (valid) Fo[(size_t)c * G + p] = v;
            }
        }
        R tot = grp_sum<G, R>(f);
        if (valid && p == 0) {
            double ll;
            int st;
            if (*m.perr) {
                ll = __builtin_nan("");
                st = 4;
            } else if (bad || isnan(logS)) {
                ll = __builtin_nan("");
                st = 2;
            } else if (!(tot > (R)0) || isinf(logS)) {
                ll = -__builtin_inf();
                st = 1;
            } else {
                ll = logS + (double)E * 0.69314718055994530942 + log((double)tot);
                st = 0;
            }
            loglik[b] = ll;
            status[b] = st;
        }
    } else {
        // backward: beta_{T-1} = 1, beta_{end(c-1)} = P_c beta_{end(c)}
        R gv = live ? (R)1 : (R)0;
        if (valid) Go[(size_t)(cb + nch - 1) * G + p] = gv;
        for (int s = 0; s + 1 < nmax; ++s) {
            const bool act = s + 1 < nch;
            const int c = act ? cb + nch - 1 - s : 0;
            R coef[G];
#pragma unroll
            for (int q = 0; q < G; ++q)
                coef[q] = act ? P[(size_t)c * GG + p * G + grp_src(p, q)] : (R)0;
            const int rr = act ? rexp[(size_t)c * G + p] : 0;
            R v = grp_dot<G, R>(gv, coef);
            const int ce = (v > (R)0) ? fexp(v) + rr : NEG_EXP;
            const int Rm = grp_max_i<G>(ce);
            v = (v > (R)0) ? fldexp(v, rr - Rm) : (R)0;
            if (act) {
                gv = v;
                if (valid) Go[(size_t)(c - 1) * G + p] = v;
            }
        }
    }
}

// ---------------------------------------------------------------- phase 3
template <typename R, int G, int L, int FAM, bool WG>
__global__ __launch_bounds__(BLOCK) void k_chunk_stats(ChunkGeom g, StagedModel<R> m,
                                                       const R *__restrict__ Fi,
                                                       const R *__restrict__ Gi,
                                                       const int32_t *__restrict__ status,
                                                       double *__restrict__ partial,
                                                       R *__restrict__ gamma_out, int64_t S) {
    constexpr int K = fam_k<FAM>();
    constexpr int KK = K > 0 ? K : 1;
    constexpr int GPW = 64 / G, GPB = (BLOCK / 64) * GPW;
    constexpr int NV = G + 2 + K;
    __shared__ double red[GPB][G][NV];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane / G, p = lane % G, grp = wave * GPW + sub;
    const int N = m.N;
    const bool live = p < N;
    using ET = typename EmitTraits<FAM, R>::T;
    const StateConsts<ET> k = load_consts(consts_ptr<FAM, R>(m), p, live);
    R coefC[G], coefR[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
        int i = grp_src(p, q);
        coefC[q] = (live && i < N) ? m.A[i * N + p] : (R)0;
        coefR[q] = (live && i < N) ? m.A[p * N + i] : (R)0;
    }
    const R pi_p = live ? m.pi[p] : (R)0;

    double xacc[G], g1acc = 0.0, gsacc = 0.0, facc[KK];
#pragma unroll
    for (int q = 0; q < G; ++q) xacc[q] = 0.0;
#pragma unroll
    for (int q = 0; q < KK; ++q) facc[q] = 0.0;

    const int per_round = gridDim.x * GPB;
    const int nrounds = (g.C + per_round - 1) / per_round;
    for (int rnd = 0; rnd < nrounds; ++rnd) {
        const int c = (rnd * (int)gridDim.x + (int)blockIdx.x) * GPB + grp;
        const bool valid = c < g.C;
        int t0 = 0, len = 0;
        int64_t off = 0;
        bool use = false;
        if (valid) {
            int b = find_seq(g.cbase, (int)g.nseq, c);
            off = g.offsets[b];
            int T = (int)(g.offsets[b + 1] - off);
            t0 = (c - g.cbase[b]) * L;
            len = min(L, T - t0);
            use = status[b] == 0;
        }
        const int tt0 = L - len;       // the chunk occupies register slots tt0 .. L-1
        const bool first = (t0 == 0);

        R y[L], e[L], al[L];
#pragma unroll
        for (int tt = 0; tt < L; ++tt) {
            const bool act = valid && tt >= tt0;
            R v = act ? load_step<FAM, R>(g.obs, off + t0 + (tt - tt0), p, N, live) : (R)1;
            Emit<ET> em = emit_step<FAM, ET>((ET)v, k, live);
            ET mx = grp_max<G, ET>(em.ell);
            y[tt] = v;
            e[tt] = (act && em.ell != neg_inf<ET>()) ? fexp_e((R)(em.ell - mx)) : (R)0;
        }
        const R ap = (valid && !first) ? Fi[(size_t)(c - 1) * G + p] : (R)0;

        // forward inside the chunk from its boundary
#pragma unroll
        for (int tt = 0; tt < L; ++tt) {
            const R xin = (tt == tt0 || tt == 0) ? ap : al[tt > 0 ? tt - 1 : 0];
            R v = e[tt] * grp_dot<G, R>(xin, coefC);
            if (first && tt == tt0) v = pi_p * e[tt];
            int ex = fexp(grp_max<G, R>(v));
            al[tt] = fldexp(v, -ex);
        }

        R U[G], gs = (R)0, g1 = (R)0, fa[KK];
#pragma unroll
        for (int q = 0; q < G; ++q) U[q] = (R)0;
#pragma unroll
        for (int q = 0; q < KK; ++q) fa[q] = (R)0;

        R bcur = valid ? Gi[(size_t)c * G + p] : (R)0;
        {   // gamma at the chunk's last step
            R h = al[L - 1] * bcur;
            R Z = grp_sum<G, R>(h);
            R gm = h * frcp(Z);
            const int tg = t0 + len - 1;
            if (use && live) {
                gs += gm;
                if constexpr (K > 0) fam_accumulate<FAM, R, KK>(gm, y[L - 1], k, fa);
                if (tg == 0) g1 += gm;
                if constexpr (WG) gamma_out[(off + tg) * N + p] = gm;
            }
        }
#pragma unroll
        for (int tt = L - 1; tt >= 0; --tt) {
            const bool trans = (tt > tt0) || (tt == tt0 && !first);
            R w = e[tt] * bcur;
            R bp = grp_dot<G, R>(w, coefR);
            const R xprev = (tt == tt0 || tt == 0) ? ap : al[tt > 0 ? tt - 1 : 0];
            R h = xprev * bp;
            R Z = grp_sum<G, R>(h);
            R rz = frcp(Z);
            const bool acc = use && trans;
            R wr = acc ? w * rz : (R)0;
            grp_outer_acc<G, R>(xprev, wr, U);
            if (tt > 0) {
                if (use && live && tt > tt0) {
                    R gm = h * rz;
                    const int tg = t0 + (tt - 1 - tt0);
                    gs += gm;
                    if constexpr (K > 0) fam_accumulate<FAM, R, KK>(gm, y[tt - 1], k, fa);
                    if (tg == 0) g1 += gm;
                    if constexpr (WG) gamma_out[(off + tg) * N + p] = gm;
                }
            }
            int ex = fexp(grp_max<G, R>(bp));
            if (trans) bcur = fldexp(bp, -ex);
        }
        if (use && live) {
#pragma unroll
            for (int q = 0; q < G; ++q) xacc[q] += (double)(U[q] * coefC[q]);
            gsacc += (double)gs;
            g1acc += (double)g1;
#pragma unroll
            for (int q = 0; q < KK; ++q) facc[q] += (double)fa[q];
        }
    }

    // fixed-order reduction over the block's lane groups
#pragma unroll
    for (int q = 0; q < G; ++q) red[grp][p][q] = xacc[q];
    red[grp][p][G] = g1acc;
    red[grp][p][G + 1] = gsacc;
#pragma unroll
    for (int q = 0; q < K; ++q) red[grp][p][G + 2 + q] = facc[q];
    __syncthreads();
    for (int64_t s = 1 + threadIdx.x; s < S; s += BLOCK) {
        int pp, slot;
        if (s <= N) {
            pp = (int)(s - 1);
            slot = G;
        } else if (s < 1 + N + (int64_t)N * N) {
            int q = (int)(s - 1 - N);
            int i = q / N, j = q % N;
            pp = j;
            slot = grp_inv(j, i);
        } else if (s < 1 + 2 * N + (int64_t)N * N) {
            pp = (int)(s - 1 - N - (int64_t)N * N);
            slot = G + 1;
        } else {
            int q = (int)(s - 1 - 2 * N - (int64_t)N * N);
            pp = q / (K > 0 ? K : 1);
            slot = G + 2 + q % (K > 0 ? K : 1);
        }
        double acc = 0.0;
        for (int gi = 0; gi < GPB; ++gi) acc += red[gi][pp][slot];
        partial[(int64_t)blockIdx.x * S + s] = acc;
    }
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * S] = 0.0;
}

// ---------------------------------------------------------------- host side
template <typename R, int G, int FAM, int L>
static void launch_phase3(int nblk, const ChunkGeom &geom, const StagedModel<R> &m, const R *F,
                          const R *Gb, const int32_t *status, double *partial, R *gamma_out,
                          int64_t S, hipStream_t s) {
    ProfScope ps("chunk_stats", s);
    if (gamma_out)
        hipLaunchKernelGGL((k_chunk_stats<R, G, L, FAM, true>), dim3(nblk), dim3(BLOCK), 0, s,
                           geom, m, F, Gb, status, partial, gamma_out, S);
    else
        hipLaunchKernelGGL((k_chunk_stats<R, G, L, FAM, false>), dim3(nblk), dim3(BLOCK), 0, s,
                           geom, m, F, Gb, status, partial, gamma_out, S);
}

template <typename R, int G, int FAM>
static hmm_status run_chunked_g(const StagedModel<R> &m, const ObsDesc &o, const ChunkBuffers &cb,
                                double *loglik, int32_t *status, R *gamma_out, double *stats,
                                int64_t S, hipStream_t s) {
    ChunkGeom geom{o.nseq, o.offsets, cb.cbase, cb.L, cb.C, ObsRef{o.obs, o.obs_f64}};
    constexpr int CPB = (BLOCK / 64) * (64 / (G * G));
    constexpr int SPB = (BLOCK / 64) * (64 / G);
    R *P = (R *)cb.P;
    R *F = (R *)cb.F;
    R *Gb = (R *)cb.Gb;
    {
        ProfScope ps("chunk_product", s);
        hipLaunchKernelGGL((k_chunk_product<R, G, FAM>), dim3((cb.C + CPB - 1) / CPB), dim3(BLOCK),
                           0, s, geom, m, P, cb.rexp, cb.clog);
    }
    {
        ProfScope ps("chunk_scan", s);
        hipLaunchKernelGGL((k_chunk_scan<R, G, FAM>), dim3((unsigned)((o.nseq + SPB - 1) / SPB), 2),
                           dim3(BLOCK), 0, s, geom, m, (const R *)P, (const int *)cb.rexp,
                           (const double *)cb.clog, F, Gb, loglik, status);
    }
    switch (cb.L) {
    case 16:
        launch_phase3<R, G, FAM, 16>(cb.nblk_stats, geom, m, F, Gb, status, cb.partial, gamma_out,
                                     S, s);
        break;
    case 32:
        launch_phase3<R, G, FAM, 32>(cb.nblk_stats, geom, m, F, Gb, status, cb.partial, gamma_out,
                                     S, s);
        break;
    case 64:
        if constexpr (sizeof(R) == 4) {
            launch_phase3<R, G, FAM, 64>(cb.nblk_stats, geom, m, F, Gb, status, cb.partial,
                                         gamma_out, S, s);
            break;
        } else {
            return HMM_ERR_UNSUPPORTED;
        }
    default:
        return HMM_ERR_UNSUPPORTED;
    }
    if (stats)
        launch_reduce_stats(cb.partial, cb.nblk_stats, S, loglik, status, o.nseq, stats, s);
    return HMM_OK;
}

template <typename R, int G>
static hmm_status run_chunked_fam(const StagedModel<R> &m, const ObsDesc &o,
                                  const ChunkBuffers &cb, double *loglik, int32_t *status,
                                  R *gamma_out, double *stats, int64_t S, hipStream_t s) {
    switch (m.family) {
    case HMM_GAUSSIAN:
        return run_chunked_g<R, G, HMM_GAUSSIAN>(m, o, cb, loglik, status, gamma_out, stats, S, s);
    case HMM_GAMMA:
        return run_chunked_g<R, G, HMM_GAMMA>(m, o, cb, loglik, status, gamma_out, stats, S, s);
    case HMM_STUDENT_T:
        return run_chunked_g<R, G, HMM_STUDENT_T>(m, o, cb, loglik, status, gamma_out, stats, S, s);
    case HMM_POISSON:
        return run_chunked_g<R, G, HMM_POISSON>(m, o, cb, loglik, status, gamma_out, stats, S, s);
    case HMM_TABLE:
        return run_chunked_g<R, G, HMM_TABLE>(m, o, cb, loglik, status, gamma_out, stats, S, s);
    default:
        return HMM_ERR_UNSUPPORTED;
    }
}

template <typename R>
hmm_status run_chunked(const StagedModel<R> &m, const ObsDesc &o, const ChunkBuffers &cb,
                       double *loglik, int32_t *status, void *gamma_out, double *stats,
                       int64_t S, hipStream_t s) {
    if (cb.G == 4)
        return run_chunked_fam<R, 4>(m, o, cb, loglik, status, (R *)gamma_out, stats, S, s);
    if (cb.G == 8)
        return run_chunked_fam<R, 8>(m, o, cb, loglik, status, (R *)gamma_out, stats, S, s);
    return HMM_ERR_UNSUPPORTED;
}

template hmm_status run_chunked<float>(const StagedModel<float> &, const ObsDesc &,
                                       const ChunkBuffers &, double *, int32_t *, void *,
                                       double *, int64_t, hipStream_t);
template hmm_status run_chunked<double>(const StagedModel<double> &, const ObsDesc &,
                                        const ChunkBuffers &, double *, int32_t *, void *,
                                        double *, int64_t, hipStream_t);

}  // namespace hmmk
